// Learned vertex ordering for the speculative colouring.
//
// Greedy first-fit uses a number of colours that depends on the vertex order;
// smallest-last order (Matula and Beck) is a good but sequential order.  A
// small MLP predicts, from local degree features, each vertex's normalised
// position in the smallest-last order; its scores become priority keys
// (lower score = coloured earlier, ties by vertex id) for color_graph.
//
// Kernels:
//   k_features     8 raw features per vertex (one group of lanes per vertex)
//   k_feat_stats   per-feature sum and sum of squares of log1p(feature)
//   k_mlp_forward  score per vertex: x = (log1p(f) - mean) / std,
//                  y = W3 relu(W2 relu(W1 x + b1) + b2) + b3, weights in BF16
//                  (stored as bf16 bits), FP32 accumulation; the 64x64 layer
//                  on matrix cores (v_mfma_f32_16x16x32_bf16)
//   k_mlp_backward per-workgroup partial gradients of the mean squared error
//                  over a minibatch (same BF16 weights in the forward part)
//   k_grad_reduce  sums the partials
//   k_adam         Adam update of the FP32 master weights, refresh of the
//                  BF16 copies
//   k_score_keys   order-preserving float -> uint32 map
// Host: exact smallest-last ranks (the training targets), bucket queue with
// per-degree min-heaps so ties go to the smallest id.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <queue>
#include <thread>
#include <vector>

#include "gcolor.h"

namespace {

constexpr int kF = GCOLOR_MLP_FEATURES;  // 8
constexpr int kH = GCOLOR_MLP_HIDDEN;    // 64
constexpr int kNP = GCOLOR_MLP_NPARAM;   // 4801
constexpr int kPW1 = GCOLOR_MLP_W1, kPB1 = GCOLOR_MLP_B1, kPW2 = GCOLOR_MLP_W2, kPB2 = GCOLOR_MLP_B2;
constexpr int kPW3 = GCOLOR_MLP_W3, kPB3 = GCOLOR_MLP_B3;
constexpr int kWedges = 8;

// ---------------------------------------------------------------------------
// Features
// ---------------------------------------------------------------------------

// splitmix64 output mix (Steele, Lea, Flood 2014): wedge choices are a pure
// function of (seed, vertex, sample index).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ bool has_edge(const int* __restrict__ row_ptr, const int* __restrict__ col, int a, int b) {
    int lo = row_ptr[a], hi = row_ptr[a + 1];
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        const int c = col[mid];
        if (c < b) lo = mid + 1;
        else if (c > b) hi = mid;
        else return true;
    }
    return false;
}

// Features (float, raw):
//  0 degree            1 log2(1 + degree)
//  2 min neighbour degree   3 mean neighbour degree   4 max neighbour degree
//  5 two-hop paths: sum over neighbours of (degree - 1)
//  6 triangle estimate: closed fraction of 8 hashed wedges * deg (deg-1) / 2
//  7 core estimate: kCoreSteps applications of the H operator to the
//    degrees (the first is the h-index of the neighbour degrees)
//
// Vertices below kFeatHeavy neighbours take a group of 8 lanes; the others
// are appended to a list and take a whole workgroup each (k_features_heavy),
// so that one hub row does not serialise the launch.
constexpr int kFeatHeavy = 128;
constexpr int kHistBins = 4096;


__device__ __forceinline__ uint64_t wedge_hash(uint64_t seed, int v, int i) {
    return mix64(seed * 0x9E3779B97F4A7C15ULL + mix64((uint64_t)v * 8ULL + (uint64_t)i + 1ULL));
}

// Sample i of vertex v (degree d >= 2, row at s): 1 if the wedge closes.
// The edge test searches the shorter of the two endpoints' rows (the
// adjacency is symmetric, so either answers it).
__device__ __forceinline__ int wedge_closed(const int* __restrict__ row_ptr, const int* __restrict__ col, int v,
                                            int s, int d, int i, uint64_t seed) {
    const uint64_t h = wedge_hash(seed, v, i);
    const int a = (int)((h & 0xffffffffULL) % (uint64_t)d);
    int b = (int)((h >> 32) % (uint64_t)(d - 1));
    if (b >= a) b += 1;
    const int wa = col[s + a], wb = col[s + b];
    const int da = row_ptr[wa + 1] - row_ptr[wa], db = row_ptr[wb + 1] - row_ptr[wb];
    return (db < da ? has_edge(row_ptr, col, wb, wa) : has_edge(row_ptr, col, wa, wb)) ? 1 : 0;
}

__device__ __forceinline__ void write_features(float* __restrict__ out, int v, int d, int mn, int mx, long long sum,
                                               int closed, int h) {
    float* f = out + (size_t)v * kF;
    f[0] = (float)d;
    f[1] = log2f(1.0f + (float)d);
    f[2] = d ? (float)mn : 0.0f;
    f[3] = d ? (float)((double)sum / (double)d) : 0.0f;
    f[4] = (float)mx;
    f[5] = (float)(sum - d);
    f[6] = d >= 2 ? (float)((double)closed / kWedges * 0.5 * (double)d * (double)(d - 1)) : 0.0f;
    f[7] = (float)h;
}

// One vertex of degree < kFeatHeavy per group of GS lanes; the neighbour
// degrees (at most kFeatHeavy / GS per lane) stay in registers.
// h-index of the values a group of GS lanes holds (kPer each, -1 for
// absent entries): the largest h with at least h values >= h.  h is at most
// cap (the count and the largest value); binary search over [0, cap].
template <int GS, int kPer>
__device__ __forceinline__ int group_h_index(const int (&x)[kPer], int cap) {
    int lo = 0, hi = cap;
    while (lo < hi) {
        const int h = (lo + hi + 1) >> 1;
        int c = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) c += x[j] >= h;
#pragma unroll
        for (int o = GS / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, GS);
        if (c >= h) lo = h;
        else hi = h - 1;
    }
    return lo;
}

template <int GS>
__device__ void features_light(int v, int s, int e, int lig, const int* __restrict__ row_ptr,
                               const int* __restrict__ col, uint64_t seed, float* __restrict__ out) {
    constexpr int kPer = kFeatHeavy / GS;
    const int d = e - s;
    int dv[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int p = s + lig + j * GS;
        dv[j] = p < e ? col[p] : -1;
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) dv[j] = dv[j] >= 0 ? row_ptr[dv[j] + 1] - row_ptr[dv[j]] : -1;
    int mn = 0x7fffffff, mx = 0;
    long long sum = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j)
        if (dv[j] >= 0) {
            mn = min(mn, dv[j]);
            mx = max(mx, dv[j]);
            sum += dv[j];
        }
#pragma unroll
    for (int o = GS / 2; o > 0; o >>= 1) {
        mn = min(mn, __shfl_xor(mn, o, GS));
        mx = max(mx, __shfl_xor(mx, o, GS));
        sum += __shfl_xor(sum, o, GS);
    }
    const int lo = group_h_index<GS, kPer>(dv, min(d, mx));
    int closed = 0;
    if (d >= 2)
        for (int i = lig; i < kWedges; i += GS) closed += wedge_closed(row_ptr, col, v, s, d, i, seed);
#pragma unroll
    for (int o = GS / 2; o > 0; o >>= 1) closed += __shfl_xor(closed, o, GS);
    if (lig == 0) write_features(out, v, d, mn, mx, sum, closed, lo);
}

__global__ __launch_bounds__(256) void k_features(int n, const int* __restrict__ row_ptr,
                                                  const int* __restrict__ col, uint64_t seed,
                                                  float* __restrict__ out, int* __restrict__ heavy,
                                                  int* __restrict__ heavy_count) {
    // 8 lanes per vertex covers the sampled wedges in one pass
    constexpr int GS = 8;
    const int groups = gridDim.x * (256 / GS);
    const int lig = threadIdx.x & (GS - 1);
    const int lane = threadIdx.x & 63;
    for (int v = blockIdx.x * (256 / GS) + threadIdx.x / GS; v < n; v += groups) {
        const int s = row_ptr[v], e = row_ptr[v + 1];
        const bool big = e - s >= kFeatHeavy;
        // wave-aggregated append of the heavy vertices (one lane per group)
        const bool app = big && lig == 0;
        const unsigned long long m = __ballot(app);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            int base = 0;
            if (lane == leader) base = atomicAdd(heavy_count, __popcll(m));
            base = __shfl(base, leader);
            if (app) heavy[base + __popcll(m & ((1ull << lane) - 1ull))] = v;
        }
        if (!big) features_light<GS>(v, s, e, lig, row_ptr, col, seed, out);
    }
}

struct HeavyLds {
    int hist[kHistBins];
    int scan[256];
    int wi[4], wj[4];
    long long wl[4];
};

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Block-wide sum / max over 256 threads (every thread gets the result).
__device__ int block_sum(HeavyLds* L, int x) {
    x = wave_sum(x);
    if ((threadIdx.x & 63) == 0) L->wi[threadIdx.x >> 6] = x;
    __syncthreads();
    const int r = L->wi[0] + L->wi[1] + L->wi[2] + L->wi[3];
    __syncthreads();
    return r;
}

__device__ int block_max(HeavyLds* L, int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    if ((threadIdx.x & 63) == 0) L->wi[threadIdx.x >> 6] = x;
    __syncthreads();
    const int r = max(max(L->wi[0], L->wi[1]), max(L->wi[2], L->wi[3]));
    __syncthreads();
    return r;
}

// h-index of the values val(col[p]) over the row [s, e), by a workgroup of
// 256 threads, with cap >= the answer (the row length and the largest value
// bound it).  It lies in [lo, hi] with f(lo) >= lo, where f(k) = number of
// entries with value >= k.  One pass over the row histograms the (clamped)
// values in [lo, hi] into at most kHistBins buckets of width W; the largest
// bucket start k with f(k) >= k narrows the range to that bucket, and width 1
// gives h exactly (at most three passes for any 32-bit value, one when the
// range is below kHistBins).  Every thread returns h.
template <class Val>
__device__ int block_h_index(HeavyLds* L, const int* __restrict__ col, int s, int e, int cap, Val val) {
    const int tid = threadIdx.x;
    int lo = 0, hi = cap;
    for (;;) {
        const int span = hi - lo + 1;
        const int W = (span + kHistBins - 1) / kHistBins;
        const int nb = (span + W - 1) / W;
        for (int j = tid; j < nb; j += 256) L->hist[j] = 0;
        __syncthreads();
        int above = 0;
        for (int p = s + tid; p < e; p += 256) {
            const int c = min(val(col[p]), cap);
            if (c > hi) ++above;
            else if (c >= lo) atomicAdd(&L->hist[(c - lo) / W], 1);
        }
        above = block_sum(L, above);  // its barrier also completes the histogram
        // thread t owns buckets [t * per, min(nb, (t + 1) * per))
        const int per = (nb + 255) / 256;
        const int j0 = min(nb, tid * per), j1 = min(nb, j0 + per);
        int cs = 0;
        for (int j = j0; j < j1; ++j) cs += L->hist[j];
        // inclusive suffix sums of the chunk sums (Hillis-Steele)
        L->scan[tid] = cs;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const int add = tid + o < 256 ? L->scan[tid + o] : 0;
            __syncthreads();
            L->scan[tid] += add;
            __syncthreads();
        }
        int run = above + L->scan[tid] - cs;  // entries in later chunks or above hi
        int best = -1;
        for (int j = j1 - 1; j >= j0; --j) {
            run += L->hist[j];
            if (run >= lo + j * W) {
                best = j;
                break;
            }
        }
        best = block_max(L, best);
        lo += best * W;
        if (W == 1) break;
        hi = min(hi, lo + W - 1);
    }
    return lo;
}

// One vertex of degree >= kFeatHeavy per workgroup of 256 threads.
__device__ void features_heavy(HeavyLds* L, int v, const int* __restrict__ row_ptr, const int* __restrict__ col,
                               uint64_t seed, float* __restrict__ out) {
    const int tid = threadIdx.x;
    const int s = row_ptr[v], e = row_ptr[v + 1];
    const int d = e - s;
    int mn = 0x7fffffff, mx = 0;
    long long sum = 0;
    for (int p = s + tid; p < e; p += 256) {
        const int w = col[p];
        const int dw = row_ptr[w + 1] - row_ptr[w];
        mn = min(mn, dw);
        mx = max(mx, dw);
        sum += dw;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn = min(mn, __shfl_xor(mn, o));
        mx = max(mx, __shfl_xor(mx, o));
        sum += __shfl_xor(sum, o);
    }
    if ((tid & 63) == 0) {
        L->wi[tid >> 6] = mn;
        L->wj[tid >> 6] = mx;
        L->wl[tid >> 6] = sum;
    }
    __syncthreads();
    mn = min(min(L->wi[0], L->wi[1]), min(L->wi[2], L->wi[3]));
    mx = max(max(L->wj[0], L->wj[1]), max(L->wj[2], L->wj[3]));
    sum = L->wl[0] + L->wl[1] + L->wl[2] + L->wl[3];
    __syncthreads();

    const int lo = block_h_index(L, col, s, e, min(d, mx),
                                 [row_ptr](int w) { return row_ptr[w + 1] - row_ptr[w]; });
    int closed = 0;
    if (tid < 64) {
        if (tid < kWedges) closed = wedge_closed(row_ptr, col, v, s, d, tid, seed);
        closed = wave_sum(closed);
    }
    if (tid == 0) write_features(out, v, d, mn, mx, sum, closed, lo);
}

__global__ __launch_bounds__(256) void k_features_heavy(const int* __restrict__ row_ptr,
                                                        const int* __restrict__ col, uint64_t seed,
                                                        const int* __restrict__ heavy,
                                                        const int* __restrict__ heavy_count,
                                                        float* __restrict__ out) {
    __shared__ HeavyLds L;
    const int total = *heavy_count;
    for (int i = blockIdx.x; i < total; i += gridDim.x) {
        features_heavy(&L, heavy[i], row_ptr, col, seed, out);
        __syncthreads();  // LDS reuse by the next vertex
    }
}

// ---------------------------------------------------------------------------
// Core estimate: the H operator (h-index of the neighbours' values) applied
// kCoreSteps times to the degrees (Lu et al., "The H-index of a network
// node and its relation to degree and coreness", 2016: the sequence falls
// monotonically to the coreness).  Step 1 is the h-index of the neighbour
// degrees that the feature kernels compute; each further step reads the
// previous step's values.  Light vertices (degree < kFeatHeavy) take 8
// lanes with the values in registers; heavy ones reuse the feature kernels'
// list and take a workgroup each with the same histogram refinement.
// ---------------------------------------------------------------------------
constexpr int kCoreSteps = 4;

__global__ __launch_bounds__(256) void k_hstep(int n, const int* __restrict__ row_ptr, const int* __restrict__ col,
                                               const int* __restrict__ hin, int* __restrict__ hout) {
    constexpr int GS = 8;
    constexpr int kPer = kFeatHeavy / GS;
    const int groups = gridDim.x * (256 / GS);
    const int lig = threadIdx.x & (GS - 1);
    for (int v = blockIdx.x * (256 / GS) + threadIdx.x / GS; v < n; v += groups) {
        const int s = row_ptr[v], e = row_ptr[v + 1];
        const int d = e - s;
        if (d >= kFeatHeavy) continue;  // the heavy kernel's vertex (the whole group skips it)
        int hv[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int q = s + lig + j * GS;
            hv[j] = q < e ? col[q] : -1;
        }
        int mx = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            hv[j] = hv[j] >= 0 ? hin[hv[j]] : -1;
            mx = max(mx, hv[j]);
        }
#pragma unroll
        for (int o = GS / 2; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, GS));
        const int h = group_h_index<GS, kPer>(hv, min(d, mx));
        if (lig == 0) hout[v] = h;
    }
}

__global__ __launch_bounds__(256) void k_hstep_heavy(const int* __restrict__ row_ptr, const int* __restrict__ col,
                                                     const int* __restrict__ heavy,
                                                     const int* __restrict__ heavy_count,
                                                     const int* __restrict__ hin, int* __restrict__ hout) {
    __shared__ HeavyLds L;
    const int total = heavy_count[0];
    // every value is at most the largest first-step value (the H sequence
    // never rises), so that bounds the search with no pass for the row's
    // largest value: one histogram pass of width 1 while it is below
    // kHistBins
    const int bound = heavy_count[1];
    for (int i = blockIdx.x; i < total; i += gridDim.x) {
        const int v = heavy[i];
        const int s = row_ptr[v], e = row_ptr[v + 1];
        const int h = block_h_index(&L, col, s, e, min(e - s, bound), [hin](int w) { return hin[w]; });
        if (threadIdx.x == 0) hout[v] = h;
        __syncthreads();  // LDS reuse by the next vertex
    }
}

// The first step's values from the feature array (and their largest value
// into *hmax), the last step's into it.
__global__ __launch_bounds__(256) void k_core_in(int n, const float* __restrict__ feat, int* __restrict__ h,
                                                 int* __restrict__ hmax) {
    __shared__ int wm[4];
    int mx = 0;
    for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
        const int x = (int)feat[(size_t)v * kF + 7];
        h[v] = x;
        mx = max(mx, x);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(hmax, max(max(wm[0], wm[1]), max(wm[2], wm[3])));
}

__global__ __launch_bounds__(256) void k_core_out(int n, const int* __restrict__ h, float* __restrict__ feat) {
    for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) feat[(size_t)v * kF + 7] = (float)h[v];
}

__global__ void k_zero_count(int* c) {
    if (threadIdx.x < 2) c[threadIdx.x] = 0;  // heavy-list length, largest first-step core estimate
}

// Per-feature sum and sum of squares of log1p(feature), in double.
__global__ __launch_bounds__(256) void k_feat_stats(int64_t n, const float* __restrict__ feat,
                                                    double* __restrict__ acc /*[2*kF]*/) {
    double s[kF], q[kF];
#pragma unroll
    for (int f = 0; f < kF; ++f) s[f] = q[f] = 0.0;
    for (int64_t v = blockIdx.x * 256LL + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
#pragma unroll
        for (int f = 0; f < kF; ++f) {
            const double x = log1p((double)feat[v * kF + f]);
            s[f] += x;
            q[f] += x * x;
        }
    }
#pragma unroll
    for (int f = 0; f < kF; ++f) {
        for (int o = 32; o > 0; o >>= 1) {
            s[f] += __shfl_xor(s[f], o);
            q[f] += __shfl_xor(q[f], o);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&acc[f], s[f]);
            atomicAdd(&acc[kF + f], q[f]);
        }
    }
}

// ---------------------------------------------------------------------------
// MLP
// ---------------------------------------------------------------------------

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Round to nearest even.
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Weights the forward pass uses: BF16 copies of W1, W2, W3 widened to FP32
// in LDS; biases FP32; input normalisation (mean, 1/std).
struct MlpLds {
    float w1[kH * kF];
    float w2[kH * kH];
    float w3[kH];
    float b1[kH];
    float b2[kH];
    float b3;
    float mean[kF];
    float istd[kF];
};

__device__ void load_mlp(MlpLds* m, const float* __restrict__ master, const uint16_t* __restrict__ wbf,
                         const float* __restrict__ norm) {
    for (int i = threadIdx.x; i < kH * kF; i += blockDim.x) m->w1[i] = bf16_to_f32(wbf[kPW1 + i]);
    for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) m->w2[i] = bf16_to_f32(wbf[kPW2 + i]);
    for (int i = threadIdx.x; i < kH; i += blockDim.x) {
        m->w3[i] = bf16_to_f32(wbf[kPW3 + i]);
        m->b1[i] = master[kPB1 + i];
        m->b2[i] = master[kPB2 + i];
    }
    if (threadIdx.x < kF) {
        m->mean[threadIdx.x] = norm[threadIdx.x];
        m->istd[threadIdx.x] = 1.0f / norm[kF + threadIdx.x];
    }
    if (threadIdx.x == 0) m->b3 = master[kPB3];
    __syncthreads();
}

__device__ __forceinline__ void normalise(const MlpLds* m, const float* __restrict__ raw, float* x) {
#pragma unroll
    for (int f = 0; f < kF; ++f) x[f] = (log1pf(raw[f]) - m->mean[f]) * m->istd[f];
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Forward pass, 16 vertices per wave at a time.  The 64x64 layer is a
// (16 x 64) x (64 x 64) product per tile on v_mfma_f32_16x16x32_bf16: lane l
// holds, of an A tile (16 x 32), row l % 16 and k = 8 (l / 16) + 0..7; of a B
// tile (32 x 16), column l % 16 and the same k; of the 16 x 16 result, rows
// 4 (l / 16) + 0..3 of column l % 16.  So each lane computes, in FP32, the 16
// first-layer units of its vertex (l % 16) that its A fragments need, and the
// W2 fragments (BF16, as stored) stay in registers for the whole launch.
// The first-layer activations enter the product as two BF16 parts (the
// rounded value and the rounding remainder), so the product keeps ~16
// significant bits of them; accumulation is FP32.
__global__ __launch_bounds__(256) void k_mlp_forward(int64_t n, const float* __restrict__ feat,
                                                     const float* __restrict__ master,
                                                     const uint16_t* __restrict__ wbf,
                                                     const float* __restrict__ norm, float* __restrict__ score) {
    __shared__ MlpLds m;
    load_mlp(&m, master, wbf, norm);
    const int l = threadIdx.x & 63;
    const int row = l & 15, kq = l >> 4;
    // W2 fragments: B[k][c] = W2[c][k] for output tile t (c = 16 t + row) and
    // k-step s (k = 32 s + 8 kq + e): eight consecutive BF16 of row c of W2
    bf16x8 bw[4][2];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
            bw[t][ks] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4*>(wbf + kPW2 + (16 * t + row) * kH + 32 * ks + 8 * kq));
    float w3c[4], b2c[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        w3c[t] = m.w3[16 * t + row];
        b2c[t] = m.b2[16 * t + row];
    }
    const int64_t tiles = (n + 15) >> 4;
    const int64_t wstride = (int64_t)gridDim.x * (256 / 64);
    for (int64_t tile = (int64_t)blockIdx.x * (256 / 64) + (threadIdx.x >> 6); tile < tiles; tile += wstride) {
        // re-read the first-layer weights from LDS each tile rather than
        // holding the 128 a lane uses in registers (that would leave one
        // wave per SIMD)
        __asm__ __volatile__("" ::: "memory");
        const int64_t v = tile * 16 + row;
        float raw[kF], x[kF];
        if (v < n) {
            const float4 f0 = *reinterpret_cast<const float4*>(feat + v * kF);
            const float4 f1 = *reinterpret_cast<const float4*>(feat + v * kF + 4);
            raw[0] = f0.x; raw[1] = f0.y; raw[2] = f0.z; raw[3] = f0.w;
            raw[4] = f1.x; raw[5] = f1.y; raw[6] = f1.z; raw[7] = f1.w;
        } else {
#pragma unroll
            for (int f = 0; f < kF; ++f) raw[f] = 0.0f;
        }
        normalise(&m, raw, x);
        // first layer: units j = 32 ks + 8 kq + e of vertex `row`
        bf16x8 ahi[2], alo[2];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int j = 32 * ks + 8 * kq + e;
                float z = m.b1[j];
#pragma unroll
                for (int f = 0; f < kF; ++f) z = fmaf(m.w1[j * kF + f], x[f], z);
                const float a = fmaxf(z, 0.0f);
                const __bf16 hi = (__bf16)a;
                ahi[ks][e] = hi;
                alo[ks][e] = (__bf16)(a - (float)hi);
            }
        // second layer on matrix cores, third layer on the vector units
        float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[ks], bw[t][ks], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[ks], bw[t][ks], acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) part[r] = fmaf(w3c[t], fmaxf(acc[r] + b2c[t], 0.0f), part[r]);
        }
        // sum over the 16 columns held by the lanes of this quarter-wave
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) part[r] += __shfl_xor(part[r], o, 16);
        if (row == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t u = tile * 16 + 4 * kq + r;
                if (u < n) score[u] = part[r] + m.b3;
            }
        }
    }
}

// Backward over a minibatch of vertices idx[0..B): per workgroup, tiles of
// 32 vertices, 8 threads per vertex for the per-vertex passes; gradient sums
// over the workgroup's vertices kept in registers, written as one partial
// row per workgroup.  Loss = mean over the minibatch of (y - target)^2.
constexpr int kTile = 32;
constexpr int kTpv = 256 / kTile;  // threads per vertex
constexpr int kUpt = kH / kTpv;    // hidden units per thread

struct BwdLds {
    MlpLds m;
    float x[kTile][kF];
    float a1[kTile][kH];
    float a2[kTile][kH];
    float dz2[kTile][kH];
    float dz1[kTile][kH];
    float dy[kTile];
    float lsum[256];
};

__global__ __launch_bounds__(256) void k_mlp_backward(int B, const int* __restrict__ idx, const float* __restrict__ feat,
                                                      const float* __restrict__ target,
                                                      const float* __restrict__ master,
                                                      const uint16_t* __restrict__ wbf,
                                                      const float* __restrict__ norm, float* __restrict__ partial,
                                                      int tiles_per_block) {
    __shared__ BwdLds L;
    load_mlp(&L.m, master, wbf, norm);
    const int t = threadIdx.x;
    const int tv = t / kTpv, tq = t % kTpv;  // vertex slot and unit slice of the per-vertex passes
    // gradient entries owned by this thread, summed over the block's tiles:
    //  dW2 row j2, columns i2 .. i2+15; dW1 entries 2t, 2t+1; unit t < 64 of
    //  db1, db2, dW3; db3 and the loss at thread 0
    float gw2[16], gw1[2] = {0.f, 0.f}, gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, loss = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) gw2[i] = 0.f;
    const int j2 = t / 4, i2 = 16 * (t % 4);
    const float invB = 1.0f / (float)B;
    for (int tile = 0; tile < tiles_per_block; ++tile) {
        const int base = (blockIdx.x * tiles_per_block + tile) * kTile;
        if (base >= B) break;  // uniform over the block
        const int slot = base + tv;
        const bool live = slot < B;
        const int v = live ? idx[slot] : 0;
        if (tq == 0) {
            float x[kF];
            if (live) normalise(&L.m, feat + (int64_t)v * kF, x);
#pragma unroll
            for (int f = 0; f < kF; ++f) L.x[tv][f] = live ? x[f] : 0.0f;
        }
        __syncthreads();
        // layer 1, this thread's units
#pragma unroll 1
        for (int u = 0; u < kUpt; ++u) {
            const int i = tq * kUpt + u;
            float z = L.m.b1[i];
#pragma unroll
            for (int f = 0; f < kF; ++f) z = fmaf(L.m.w1[i * kF + f], L.x[tv][f], z);
            L.a1[tv][i] = fmaxf(z, 0.0f);
        }
        __syncthreads();
        // layer 2 and this thread's share of the output
        float yp = 0.f;
#pragma unroll 1
        for (int u = 0; u < kUpt; ++u) {
            const int j = tq * kUpt + u;
            float z = L.m.b2[j];
#pragma unroll 8
            for (int i = 0; i < kH; ++i) z = fmaf(L.m.w2[j * kH + i], L.a1[tv][i], z);
            const float a = fmaxf(z, 0.0f);
            L.a2[tv][j] = a;
            yp = fmaf(L.m.w3[j], a, yp);
        }
#pragma unroll
        for (int o = kTpv / 2; o > 0; o >>= 1) yp += __shfl_xor(yp, o, kTpv);
        if (tq == 0) {
            const float r = live ? yp + L.m.b3 - target[v] : 0.0f;
            L.dy[tv] = 2.0f * r * invB;
            loss += r * r * invB;
        }
        __syncthreads();
        // dL/dz2 = dy * W3 on the active units
#pragma unroll 1
        for (int u = 0; u < kUpt; ++u) {
            const int j = tq * kUpt + u;
            L.dz2[tv][j] = L.a2[tv][j] > 0.0f ? L.dy[tv] * L.m.w3[j] : 0.0f;
        }
        __syncthreads();
        // dL/dz1 = (W2^T dz2) on the active units
#pragma unroll 1
        for (int u = 0; u < kUpt; ++u) {
            const int i = tq * kUpt + u;
            float g = 0.f;
#pragma unroll 8
            for (int j = 0; j < kH; ++j) g = fmaf(L.m.w2[j * kH + i], L.dz2[tv][j], g);
            L.dz1[tv][i] = L.a1[tv][i] > 0.0f ? g : 0.0f;
        }
        __syncthreads();
        // sums over the tile's vertices
#pragma unroll 2
        for (int b = 0; b < kTile; ++b) {
            const float dz = L.dz2[b][j2];
#pragma unroll
            for (int i = 0; i < 16; ++i) gw2[i] = fmaf(dz, L.a1[b][i2 + i], gw2[i]);
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int e = 2 * t + r, i = e / kF, f = e % kF;
            float g = 0.f;
            for (int b = 0; b < kTile; ++b) g = fmaf(L.dz1[b][i], L.x[b][f], g);
            gw1[r] += g;
        }
        if (t < kH) {
            for (int b = 0; b < kTile; ++b) {
                gb1 += L.dz1[b][t];
                gb2 += L.dz2[b][t];
                gw3 = fmaf(L.a2[b][t], L.dy[b], gw3);
            }
        }
        if (t == 0)
            for (int b = 0; b < kTile; ++b) gb3 += L.dy[b];
        __syncthreads();
    }
    // one partial row per block: kNP gradients, then the loss
    float* row = partial + (size_t)blockIdx.x * (kNP + 1);
#pragma unroll
    for (int i = 0; i < 16; ++i) row[kPW2 + j2 * kH + i2 + i] = gw2[i];
    row[kPW1 + 2 * t] = gw1[0];
    row[kPW1 + 2 * t + 1] = gw1[1];
    if (t < kH) {
        row[kPB1 + t] = gb1;
        row[kPB2 + t] = gb2;
        row[kPW3 + t] = gw3;
    }
    L.lsum[t] = loss;
    __syncthreads();
    if (t == 0) {
        float s = 0.f;
        for (int i = 0; i < 256; ++i) s += L.lsum[i];
        row[kPB3] = gb3;
        row[kNP] = s;
    }
}

__global__ __launch_bounds__(256) void k_grad_reduce(int nblocks, const float* __restrict__ partial,
                                                     float* __restrict__ grad /*[kNP + 1]*/) {
    for (int p = blockIdx.x * 256 + threadIdx.x; p <= kNP; p += gridDim.x * 256) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * (kNP + 1) + p];
        grad[p] = (float)s;
    }
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ master, uint16_t* __restrict__ wbf,
                                              float* __restrict__ mom, float* __restrict__ vel,
                                              const float* __restrict__ grad, float lr, float b1, float b2,
                                              float eps, int step) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    for (int p = blockIdx.x * 256 + threadIdx.x; p < kNP; p += gridDim.x * 256) {
        const float g = grad[p];
        const float m = b1 * mom[p] + (1.0f - b1) * g;
        const float v = b2 * vel[p] + (1.0f - b2) * g * g;
        mom[p] = m;
        vel[p] = v;
        const float w = master[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
        master[p] = w;
        wbf[p] = f32_to_bf16(w);
    }
}

__global__ __launch_bounds__(256) void k_refresh_bf16(const float* __restrict__ master, uint16_t* __restrict__ wbf) {
    for (int p = blockIdx.x * 256 + threadIdx.x; p < kNP; p += gridDim.x * 256) wbf[p] = f32_to_bf16(master[p]);
}

// Normalisation from the sums of k_feat_stats over `count` vertices: per
// feature the mean and the population standard deviation of log1p(feature),
// the variance floored at 1e-12 (a constant feature keeps a finite scale).
__global__ void k_feat_norm(int64_t count, const double* __restrict__ acc, float* __restrict__ norm) {
    const int f = threadIdx.x;
    if (f >= kF) return;
    const double c = (double)count;
    const double mean = acc[f] / c;
    const double var = fmax(acc[kF + f] / c - mean * mean, 1e-12);
    norm[f] = (float)mean;
    norm[kF + f] = (float)sqrt(var);
}

// Training target of smallest-last position r among n vertices:
// log(1 + r) / log(max(n, 2)), in [0, 1] and increasing in r.
__global__ __launch_bounds__(256) void k_rank_targets(int n, const int* __restrict__ rank, float* __restrict__ target) {
    const double inv = 1.0 / log((double)max(n, 2));
    for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256)
        target[v] = (float)(log1p((double)rank[v]) * inv);
}

// Order-preserving map of float scores to uint32 keys: flip all bits of a
// negative float, flip only the sign bit of a non-negative one.  NaN scores
// are reported through *bad.
__global__ __launch_bounds__(256) void k_score_keys(int64_t n, const float* __restrict__ score,
                                                    uint32_t* __restrict__ keys, int* bad) {
    for (int64_t v = blockIdx.x * 256LL + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
        const float s = score[v];
        if (s != s) atomicOr(bad, 1);
        const uint32_t u = __float_as_uint(s);
        keys[v] = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    }
}

// Per-device buffer for the heavy-vertex list of gcolor_features: a count
// (padded to 256 bytes) and up to n vertex ids; grown on demand.
int grid_for(int64_t items, int per_block) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    const int64_t want = (items + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)cus * 8));
}

// ---------------------------------------------------------------------------
// Host: exact smallest-last ranks
// ---------------------------------------------------------------------------

// Repeatedly remove a vertex of minimum remaining degree, the smallest id
// among those; the colouring order is the reverse removal order, rank[v] is
// v's position in it.  Buckets per degree hold min-heaps of ids with lazy
// deletion (an entry is live when its degree still matches).
int32_t smallest_last_host(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* rank) {
    std::vector<int32_t> deg(n);
    std::vector<char> gone(n, 0);
    int32_t maxd = 0;
    for (int32_t v = 0; v < n; ++v) {
        int32_t d = 0;
        for (int32_t p = row_ptr[v]; p < row_ptr[v + 1]; ++p) d += col[p] != v;
        deg[v] = d;
        maxd = std::max(maxd, d);
    }
    using Heap = std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>>;
    std::vector<Heap> bucket(maxd + 1);
    for (int32_t v = 0; v < n; ++v) bucket[deg[v]].push(v);
    int32_t cur = 0, degeneracy = 0;
    for (int32_t removed = 0; removed < n; ++removed) {
        int32_t v = -1;
        for (;;) {
            while (bucket[cur].empty()) ++cur;
            const int32_t c = bucket[cur].top();
            bucket[cur].pop();
            if (!gone[c] && deg[c] == cur) {
                v = c;
                break;
            }
        }
        gone[v] = 1;
        degeneracy = std::max(degeneracy, cur);
        rank[v] = n - 1 - removed;
        for (int32_t p = row_ptr[v]; p < row_ptr[v + 1]; ++p) {
            const int32_t w = col[p];
            if (w == v || gone[w]) continue;
            bucket[--deg[w]].push(w);
            if (deg[w] < cur) cur = deg[w];
        }
    }
    return degeneracy;
}

}  // namespace

extern "C" {

size_t gcolor_features_workspace_bytes(int32_t n) {
    if (n < 0) return 0;
    // heavy-vertex list (count + ids), then two arrays for the core-estimate steps
    return ((size_t)n + 64) * sizeof(int) + (kCoreSteps > 1 ? 2 * (size_t)n * sizeof(int) : 0);
}

int gcolor_features(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint64_t seed, float* feat_out,
                    void* workspace, size_t ws_bytes, gcolor_stream_t stream) {
    if (n < 0) return GCOLOR_EINVAL;
    if (n == 0) return GCOLOR_OK;
    if (!row_ptr || !feat_out || !workspace) return GCOLOR_EINVAL;
    if (ws_bytes < gcolor_features_workspace_bytes(n)) return GCOLOR_EWORKSPACE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int* count = static_cast<int*>(workspace);
    int* list = count + 64;
    k_zero_count<<<1, 64, 0, st>>>(count);
    k_features<<<grid_for(n, 32), 256, 0, st>>>(n, row_ptr, col_idx, seed, feat_out, list, count);
    // one workgroup per listed vertex (grid-strided over the device count)
    k_features_heavy<<<grid_for(n, kFeatHeavy), 256, 0, st>>>(row_ptr, col_idx, seed, list, count, feat_out);
    if (kCoreSteps > 1) {
        int* h0 = list + n;
        int* h1 = h0 + n;
        k_core_in<<<grid_for(n, 256), 256, 0, st>>>(n, feat_out, h0, count + 1);
        for (int step = 2; step <= kCoreSteps; ++step) {
            k_hstep<<<grid_for(n, 32), 256, 0, st>>>(n, row_ptr, col_idx, h0, h1);
            k_hstep_heavy<<<grid_for(n, kFeatHeavy), 256, 0, st>>>(row_ptr, col_idx, list, count, h0, h1);
            std::swap(h0, h1);
        }
        k_core_out<<<grid_for(n, 256), 256, 0, st>>>(n, h0, feat_out);
    }
    return hipGetLastError() == hipSuccess ? GCOLOR_OK : GCOLOR_EHIP;
}

int gcolor_feature_stats(int64_t n, const float* feat, double* acc, gcolor_stream_t stream) {
    if (n < 0 || !acc) return GCOLOR_EINVAL;
    if (n == 0) return GCOLOR_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    k_feat_stats<<<grid_for(n, 256), 256, 0, st>>>(n, feat, acc);
    return hipGetLastError() == hipSuccess ? GCOLOR_OK : GCOLOR_EHIP;
}

int gcolor_mlp_forward(int64_t n, const float* feat, const float* master, const uint16_t* wbf, const float* norm,
                       float* score, gcolor_stream_t stream) {
    if (n < 0 || !master || !wbf || !norm) return GCOLOR_EINVAL;
    if (n == 0) return GCOLOR_OK;
    if (!feat || !score) return GCOLOR_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    k_mlp_forward<<<grid_for((n + 15) / 16, 4), 256, 0, st>>>(n, feat, master, wbf, norm, score);
    return hipGetLastError() == hipSuccess ? GCOLOR_OK : GCOLOR_EHIP;
}

size_t gcolor_mlp_partial_floats(int32_t batch) {
    if (batch <= 0) return 0;
    const int tiles = (batch + kTile - 1) / kTile;
    const int tpb = std::max(1, (tiles + 511) / 512);
    const int blocks = (tiles + tpb - 1) / tpb;
    return (size_t)blocks * (kNP + 1);
}

int gcolor_mlp_grad(int32_t batch, const int32_t* idx, const float* feat, const float* target, const float* master,
                    const uint16_t* wbf, const float* norm, float* partial, float* grad, gcolor_stream_t stream) {
    if (batch <= 0 || !idx || !feat || !target || !master || !wbf || !norm || !partial || !grad)
        return GCOLOR_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int tiles = (batch + kTile - 1) / kTile;
    const int tpb = std::max(1, (tiles + 511) / 512);
    const int blocks = (tiles + tpb - 1) / tpb;
    k_mlp_backward<<<blocks, 256, 0, st>>>(batch, idx, feat, target, master, wbf, norm, partial, tpb);
    if (hipGetLastError() != hipSuccess) return GCOLOR_EHIP;
    k_grad_reduce<<<(kNP + 256) / 256, 256, 0, st>>>(blocks, partial, grad);
    return hipGetLastError() == hipSuccess ? GCOLOR_OK : GCOLOR_EHIP;
}

int gcolor_mlp_adam(float* master, uint16_t* wbf, float* mom, float* vel, const float* grad, float lr, float beta1,
                    float beta2, float eps, int32_t step, gcolor_stream_t stream) {
    if (!master || !wbf || !mom || !vel || !grad || step < 1) return GCOLOR_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    k_adam<<<(kNP + 255) / 256, 256, 0, st>>>(master, wbf, mom, vel, grad, lr, beta1, beta2, eps, step);
    return hipGetLastError() == hipSuccess ? GCOLOR_OK : GCOLOR_EHIP;
}

int gcolor_mlp_refresh_bf16(const float* master, uint16_t* wbf, gcolor_stream_t stream) {
    if (!master || !wbf) return GCOLOR_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    k_refresh_bf16<<<(kNP + 255) / 256, 256, 0, st>>>(master, wbf);
    return hipGetLastError() == hipSuccess ? GCOLOR_OK : GCOLOR_EHIP;
}

int gcolor_scores_to_keys(int64_t n, const float* score, uint32_t* keys, int32_t* bad, gcolor_stream_t stream) {
    if (n < 0 || !bad) return GCOLOR_EINVAL;
    if (n == 0) return GCOLOR_OK;
    if (!score || !keys) return GCOLOR_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    k_score_keys<<<grid_for(n, 256), 256, 0, st>>>(n, score, keys, bad);
    return hipGetLastError() == hipSuccess ? GCOLOR_OK : GCOLOR_EHIP;
}

int gcolor_feature_norm(int64_t count, const double* acc, float* norm, gcolor_stream_t stream) {
    if (count <= 0 || !acc || !norm) return GCOLOR_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    k_feat_norm<<<1, 64, 0, st>>>(count, acc, norm);
    return hipGetLastError() == hipSuccess ? GCOLOR_OK : GCOLOR_EHIP;
}

int gcolor_rank_targets(int32_t n, const int32_t* rank, float* target, gcolor_stream_t stream) {
    if (n < 0) return GCOLOR_EINVAL;
    if (n == 0) return GCOLOR_OK;
    if (!rank || !target) return GCOLOR_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    k_rank_targets<<<grid_for(n, 256), 256, 0, st>>>(n, rank, target);
    return hipGetLastError() == hipSuccess ? GCOLOR_OK : GCOLOR_EHIP;
}

size_t gcolor_order_learned_workspace_bytes(int32_t n) {
    if (n < 0) return 0;
    const size_t feat = (((size_t)n * kF * sizeof(float)) + 255) & ~(size_t)255;
    const size_t score = (((size_t)n * sizeof(float)) + 255) & ~(size_t)255;
    return feat + score + gcolor_features_workspace_bytes(n);
}

int gcolor_order_learned(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint64_t seed,
                         const float* master, const uint16_t* wbf, const float* norm, uint32_t* keys_out,
                         int32_t* nan_flag, void* workspace, size_t ws_bytes, gcolor_stream_t stream) {
    if (n < 0 || !master || !wbf || !norm || !nan_flag) return GCOLOR_EINVAL;
    if (n == 0) return GCOLOR_OK;
    if (!row_ptr || !keys_out || !workspace) return GCOLOR_EINVAL;
    if (ws_bytes < gcolor_order_learned_workspace_bytes(n)) return GCOLOR_EWORKSPACE;
    char* base = static_cast<char*>(workspace);
    float* feat = reinterpret_cast<float*>(base);
    const size_t fb = (((size_t)n * kF * sizeof(float)) + 255) & ~(size_t)255;
    float* score = reinterpret_cast<float*>(base + fb);
    const size_t sb = (((size_t)n * sizeof(float)) + 255) & ~(size_t)255;
    void* fws = base + fb + sb;
    int rc = gcolor_features(n, row_ptr, col_idx, seed, feat, fws, gcolor_features_workspace_bytes(n), stream);
    if (rc) return rc;
    rc = gcolor_mlp_forward(n, feat, master, wbf, norm, score, stream);
    if (rc) return rc;
    return gcolor_scores_to_keys(n, score, keys_out, nan_flag, stream);
}

int gcolor_smallest_last_host(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t* rank,
                              int32_t* degeneracy) {
    if (n < 0 || (n > 0 && (!row_ptr || !rank))) return GCOLOR_EINVAL;
    if (n == 0) {
        if (degeneracy) *degeneracy = 0;
        return GCOLOR_OK;
    }
    if (row_ptr[n] > 0 && !col_idx) return GCOLOR_EINVAL;
    const int32_t d = smallest_last_host(n, row_ptr, col_idx, rank);
    if (degeneracy) *degeneracy = d;
    return GCOLOR_OK;
}

}  // extern "C"
