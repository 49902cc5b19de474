// Block Gauss-Seidel variant of the speculative colouring (Algorithm 2 with
// the static schedule of the section "Scalability Results": each thread owns
// a fixed contiguous range of vertices, visits it in index order and sees
// its own colours of the current round at once).
//
// Blocks are the id ranges [b*B, (b+1)*B).  Round k, U = uncoloured vertices:
//   phase 1 (k_blk_first, one wavefront per block): the block's vertices of
//     U in ascending id take the smallest colour held neither by a coloured
//     neighbour nor by a neighbour of the same block chosen earlier in this
//     round (kept in LDS while the block is coloured, then copied to tent);
//   phase 2 (k_blk_check, one thread per vertex): v in U loses when a
//     neighbour holds its colour (tent for vertices of U, the committed
//     colour otherwise) and precedes it in (key, id) order;
//   phase 3 (k_blk_commit): winners commit, losers form U for round k+1.
// The kernel boundaries order the phases, so the result is a function of the
// input and B.  B = 1 is Algorithm 2 itself; one block holding every vertex
// is the serial greedy in index order, done in one round.  Every round
// commits the uncoloured vertex first in (key, id) order, so a graph of n
// vertices needs at most n rounds.
//
// Memory: colors_out holds the committed colours (0 = uncoloured); the
// workspace holds a 256-byte control block, tent (int32[n]) and the phase-2
// verdicts (int32[n]).  Block sizes run from 1 to kMaxBlock (LDS per
// wavefront: 4 bytes per vertex of its block).

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

struct BlkCtl {
    unsigned long long committed;  // vertices committed so far
    long long work;                // sum over rounds of the degrees of U
    int32_t rounds;                // last round that committed a vertex
    int32_t maxcolor;
    int32_t pad[58];
};
static_assert(sizeof(BlkCtl) == 256, "control block");

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct BlkLayout {
    size_t tent, win, total;
};

BlkLayout blk_layout(int32_t n) {
    BlkLayout L;
    const size_t vn = sizeof(int32_t) * (size_t)(n > 0 ? n : 1);
    L.tent = align_up(sizeof(BlkCtl));
    L.win = L.tent + align_up(vn);
    L.total = L.win + align_up(vn);
    return L;
}

__device__ __forceinline__ bool blk_before(const uint32_t* __restrict__ key, int w, int v) {
    if (!key) return w < v;
    const uint32_t kw = key[w], kv = key[v];
    return kw < kv || (kw == kv && w < v);
}

__global__ void k_blk_init(int n, int* __restrict__ color, BlkCtl* ctl) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i == 0) {
        ctl->committed = 0;
        ctl->work = 0;
        ctl->rounds = 0;
        ctl->maxcolor = 0;
    }
    for (int v = i; v < n; v += gridDim.x * kThreads) color[v] = 0;
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

// Phase 1: one wavefront per block, its uncoloured vertices in ascending id;
// the lanes stride each row (four entries per lane per step) and OR their
// masks of the colours base..base+63 they see.
__global__ __launch_bounds__(kThreads) void k_blk_first(int n, int B, long long nblocks,
                                                        const int* __restrict__ row_ptr,
                                                        const int* __restrict__ col_idx,
                                                        const int* __restrict__ color, int* __restrict__ tent) {
    extern __shared__ int lds[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int* lt = lds + wid * B;
    for (long long b = (long long)blockIdx.x * kWaves + wid; b < nblocks; b += (long long)gridDim.x * kWaves) {
        const int v0 = (int)(b * B);
        const int v1 = (int)std::min<long long>(n, (long long)v0 + B);
        for (int v = v0; v < v1; ++v) {
            if (color[v] != 0) continue;  // uniform over the wavefront
            const int s = row_ptr[v], e = row_ptr[v + 1];
            int t = 0;
            for (int base = 1; t == 0; base += 64) {
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
                if (~m) t = base + __builtin_ctzll(~m);
            }
            if (lane == 0) lt[v - v0] = t;
            wave_sync();
        }
        for (int i = lane; i < v1 - v0; i += 64)
            if (color[v0 + i] == 0) tent[v0 + i] = lt[i];
        wave_sync();  // the slot is reused by the wavefront's next block
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

// Phase 2: verdict of every uncoloured vertex against this round's colours.
__global__ __launch_bounds__(kThreads) void k_blk_check(int n, const int* __restrict__ row_ptr,
                                                        const int* __restrict__ col_idx,
                                                        const uint32_t* __restrict__ key,
                                                        const int* __restrict__ color,
                                                        const int* __restrict__ tent, int* __restrict__ win,
                                                        BlkCtl* ctl) {
    __shared__ long long red[kThreads / 64];
    long long work = 0;
    for (int v = blockIdx.x * kThreads + threadIdx.x; v < n; v += gridDim.x * kThreads) {
        if (color[v] != 0) continue;
        const int s = row_ptr[v], e = row_ptr[v + 1];
        const int tv = tent[v];
        bool lose = false;
        for (int p0 = s; p0 < e && !lose; p0 += 4) {
            int w[4], cw[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) w[j] = p0 + j < e ? col_idx[p0 + j] : v;
#pragma unroll
            for (int j = 0; j < 4; ++j) cw[j] = color[w[j]];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (w[j] != v) lose |= (cw[j] != 0 ? cw[j] : tent[w[j]]) == tv && blk_before(key, w[j], v);
        }
        win[v] = lose ? 0 : 1;
        work += e - s;
    }
    const long long t = blk_block_sum(work, red);
    if (threadIdx.x == 0 && t) atomicAdd((unsigned long long*)&ctl->work, (unsigned long long)t);
}

// Phase 3: winners commit.
__global__ __launch_bounds__(kThreads) void k_blk_commit(int n, int k, int* __restrict__ color,
                                                         const int* __restrict__ tent,
                                                         const int* __restrict__ win, BlkCtl* ctl) {
    __shared__ long long red[kThreads / 64];
    long long c = 0;
    int mx = 0;
    for (int v = blockIdx.x * kThreads + threadIdx.x; v < n; v += gridDim.x * kThreads) {
        if (color[v] != 0 || !win[v]) continue;
        color[v] = tent[v];
        mx = max(mx, tent[v]);
        ++c;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
    if ((threadIdx.x & 63) == 0 && mx) atomicMax(&ctl->maxcolor, mx);
    const long long t = blk_block_sum(c, red);
    if (threadIdx.x == 0 && t) {
        atomicAdd(&ctl->committed, (unsigned long long)t);
        atomicMax(&ctl->rounds, k);
    }
}

struct DevWs {
    void* p = nullptr;
    size_t bytes = 0;
};
std::mutex g_mu;
std::vector<DevWs> g_ws;

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

// Per-thread pinned staging for the control block.
BlkCtl* blk_host() {
    thread_local BlkCtl* h = nullptr;
    if (!h && hipHostMalloc((void**)&h, sizeof(BlkCtl), hipHostMallocDefault) != hipSuccess) h = nullptr;
    return h;
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
    BlkCtl* h = blk_host();
    if (!h) return GCOLOR_EHIP;
    BLK_CHECK(hipMemcpyAsync(&h->pad[0], row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    BLK_CHECK(hipStreamSynchronize(st));
    const int64_t nnz = h->pad[0];
    if (nnz < 0) return GCOLOR_ECSR;
    if (nnz > 0 && !col_idx) return GCOLOR_EINVAL;
    int dev = 0;
    BLK_CHECK(hipGetDevice(&dev));
    const BlkLayout L = blk_layout(n);
    void* ws = workspace;
    if (ws) {
        if (ws_bytes < L.total) return GCOLOR_EWORKSPACE;
    } else {
        const int rc = blk_workspace(dev, L.total, &ws);
        if (rc) return rc;
    }
    char* base = static_cast<char*>(ws);
    BlkCtl* ctl = reinterpret_cast<BlkCtl*>(base);
    int* tent = reinterpret_cast<int*>(base + L.tent);
    int* win = reinterpret_cast<int*>(base + L.win);
    int32_t cap = 0;
    gcolor_get_round_cap(&cap);
    const long long limit = cap > 0 ? cap : (long long)n + 64;
    const long long nblocks = ((long long)n + block_size - 1) / block_size;
    const int vgrid = grid_for(dev, n), bgrid = grid_for(dev, nblocks * 64);  // kWaves blocks per workgroup
    const size_t lds_bytes = sizeof(int) * (size_t)kWaves * (size_t)block_size;

    k_blk_init<<<vgrid, kThreads, 0, st>>>(n, colors_out, ctl);
    BLK_CHECK(hipGetLastError());
    long long k = 0;
    int batch = 4;
    int rc = GCOLOR_OK;
    for (;;) {
        const long long nb = std::min<long long>(batch, limit - k);
        for (long long j = 0; j < nb; ++j) {
            ++k;
            k_blk_first<<<bgrid, kThreads, lds_bytes, st>>>(n, block_size, nblocks, row_ptr, col_idx, colors_out,
                                                            tent);
            k_blk_check<<<vgrid, kThreads, 0, st>>>(n, row_ptr, col_idx, priority, colors_out, tent, win, ctl);
            k_blk_commit<<<vgrid, kThreads, 0, st>>>(n, (int)k, colors_out, tent, win, ctl);
            BLK_CHECK(hipGetLastError());
        }
        BLK_CHECK(hipMemcpyAsync(h, ctl, sizeof(BlkCtl), hipMemcpyDeviceToHost, st));
        BLK_CHECK(hipStreamSynchronize(st));
        if (h->committed >= (unsigned long long)n) break;
        if (k >= limit) {
            rc = GCOLOR_EROUNDS;
            break;
        }
        batch = std::min(batch * 2, 16);
    }
    if (rc == GCOLOR_OK && h->committed != (unsigned long long)n) rc = GCOLOR_EINTERNAL;
    if (stats) {
        if (rc == GCOLOR_OK) {
            stats->rounds = h->rounds;
            stats->num_colors = h->maxcolor;
            stats->edge_work = h->work;
        }
        stats->status = rc;
    }
    return rc;
}

}  // extern "C"
