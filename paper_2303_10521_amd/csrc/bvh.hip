// bvh.hip -- linear BVH over arbitrary primitive boxes.
//
// Build: Morton codes of box centroids (b bits per axis over the centroid
// bounds, b growing with the primitive count: 10 up to 2^18 primitives), LSD
// radix sort, Karras-style hierarchy emission
// (T. Karras, "Maximizing parallelism in the construction of BVHs, octrees
// and k-d trees", HPG 2012) with ties between equal codes broken by the sorted
// index, then a bottom-up refit.  Each internal node stores both child boxes,
// its parent link and the split axis (the Morton bit at which its range
// splits), which the traversal uses to visit the near child first.
// Up to four trees build in one batch: the tree number sits above the Morton
// bits, so one sort orders every tree's primitives into its own contiguous
// segment, and each later launch (emission, refit) covers all the trees.
// Refit: one thread per leaf climbs towards the root; the second thread to
// arrive at a node (device-scope acquire-release counter) merges the two
// child boxes and continues, so every node is written exactly once per refit.
// Paper: Section II-A (a BVH updated between frames), Section III-A (only
// subtrees change within a trajectory segment).
#include <algorithm>
#include <deque>
#include <math.h>
#include <string.h>

#include <utility>
#include <vector>

#include "emrt_dev.h"
#include "emrt_launch.h"

namespace emrt {

__device__ __forceinline__ uint32_t f2ord(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
    u = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    return __uint_as_float(u);
}

__device__ __forceinline__ unsigned long long split3(uint32_t a) {
    unsigned long long x = a & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}

__global__ void k_fill_zero1(uint32_t* p) { *p = 0u; }

// The trees of one batched build: tree j owns the sorted positions
// [off[j], off[j + 1]).
struct BuildSet {
    const float* box[kMaxBuildJobs];
    BNode* nodes[kMaxBuildJobs];
    int* leaf_parent[kMaxBuildJobs];
    uint32_t* perm[kMaxBuildJobs];
    uint32_t* counters[kMaxBuildJobs];
    int* span[kMaxBuildJobs];
    int off[kMaxBuildJobs + 1];
    int nj;
    int bits;  // Morton bits per axis
};

struct RefitBlocks {
    int blk[kMaxBuildJobs + 1];  // first block of each tree
};

__device__ __forceinline__ int job_of(const BuildSet& S, int i) {
    int j = 0;
    while (j + 1 < S.nj && i >= S.off[j + 1]) j++;
    return j;
}

__global__ void k_init_bounds(uint32_t* b, int nj) {
    int t = threadIdx.x;
    if (t < 6 * nj) b[t] = (t % 6) < 3 ? 0xFFFFFFFFu : 0u;
}

// centroid bounds of every tree (ordered-integer min/max), [nj][6]
__global__ void __launch_bounds__(256) k_bounds(BuildSet S, uint32_t* b) {
    __shared__ uint32_t sh[6 * kMaxBuildJobs];
    if (threadIdx.x < 6 * kMaxBuildJobs) sh[threadIdx.x] = (threadIdx.x % 6) < 3 ? 0xFFFFFFFFu : 0u;
    __syncthreads();
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S.off[S.nj]) {
        int j = job_of(S, i);
        const float* p = S.box[j] + 6 * (long long)(i - S.off[j]);
        for (int c = 0; c < 3; c++) {
            float m = 0.5f * (p[c] + p[3 + c]);
            atomicMin(&sh[6 * j + c], f2ord(m));
            atomicMax(&sh[6 * j + 3 + c], f2ord(m));
        }
    }
    __syncthreads();
    int t = threadIdx.x;
    if (t < 6 * S.nj) {
        if ((t % 6) < 3) atomicMin(&b[t], sh[t]);
        else atomicMax(&b[t], sh[t]);
    }
}

// key = tree number above 3 * bits Morton bits; value = primitive index
__global__ void __launch_bounds__(256) k_morton(BuildSet S, const uint32_t* b, unsigned long long* codes,
                                                uint32_t* vals) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.off[S.nj]) return;
    int j = job_of(S, i);
    int li = i - S.off[j];
    const float* p = S.box[j] + 6 * (long long)li;
    const float scale = (float)((1u << S.bits) - 1u);
    uint32_t q[3];
    for (int c = 0; c < 3; c++) {
        float lo = ord2f(b[6 * j + c]), hi = ord2f(b[6 * j + 3 + c]);
        float m = 0.5f * (p[c] + p[3 + c]);
        float e = hi - lo;
        float u = e > 0.0f ? (m - lo) / e : 0.5f;
        u = fminf(fmaxf(u, 0.0f), 1.0f);
        q[c] = (uint32_t)(u * scale);
    }
    codes[i] = ((unsigned long long)j << (3 * S.bits)) | (split3(q[0]) << 2) | (split3(q[1]) << 1) | split3(q[2]);
    vals[i] = (uint32_t)li;
}

__device__ __forceinline__ int kdelta(const unsigned long long* c, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    unsigned long long a = c[i], b = c[j];
    if (a == b) return 64 + __clz((uint32_t)(i ^ j));
    return __clzll((long long)(a ^ b));
}

// Internal node i of one tree over its sorted codes [n] (and its leaf slot i).
__device__ __forceinline__ void emit_node(const unsigned long long* codes, const uint32_t* sorted, int n, int i,
                                          BNode* nodes, int* leaf_parent, uint32_t* perm, int* span) {
    if (i < n) perm[i] = sorted[i];
    if (n == 1 && i == 0) {
        BNode nd;
        nd.a = make_float4(INFINITY, INFINITY, INFINITY, -INFINITY);
        nd.b = make_float4(-INFINITY, -INFINITY, INFINITY, INFINITY);
        nd.c = make_float4(INFINITY, -INFINITY, -INFINITY, -INFINITY);
        nd.m = make_int4((int)EMRT_LEAF, (int)EMRT_LEAF, -1, 0);
        nodes[0] = nd;
        leaf_parent[0] = 0;
        span[0] = 0;
        return;
    }
    if (i >= n - 1) return;
    int d = (kdelta(codes, n, i, i + 1) - kdelta(codes, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = kdelta(codes, n, i, i - d);
    int lmax = 2;
    while (kdelta(codes, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (kdelta(codes, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = kdelta(codes, n, i, j);
    int s = 0;
    int t = l;
    do {
        t = (t + 1) / 2;
        if (kdelta(codes, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int gamma = i + s * d + (d < 0 ? -1 : 0);
    span[i] = j;
    int lo = i < j ? i : j, hi = i < j ? j : i;
    int left = (lo == gamma) ? (int)(EMRT_LEAF | (uint32_t)gamma) : gamma;
    int right = (hi == gamma + 1) ? (int)(EMRT_LEAF | (uint32_t)(gamma + 1)) : gamma + 1;
    int axis = 0;
    if (dnode < 64) {
        int bit = 63 - dnode;
        int r = bit % 3;
        axis = r == 2 ? 0 : (r == 1 ? 1 : 2);
    }
    int* m = (int*)&nodes[i].m;
    m[0] = left;
    m[1] = right;
    m[3] = axis;
    if (i == 0) m[2] = -1;
    if (lo == gamma) leaf_parent[gamma] = i;
    else ((int*)&nodes[gamma].m)[2] = i;
    if (hi == gamma + 1) leaf_parent[gamma + 1] = (int)((uint32_t)i | EMRT_SIDE);
    else ((int*)&nodes[gamma + 1].m)[2] = (int)((uint32_t)i | EMRT_SIDE);
}

__global__ void __launch_bounds__(256) k_emit(BuildSet S, const unsigned long long* codes, const uint32_t* sorted) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.off[S.nj]) return;
    int j = job_of(S, i);
    int o = S.off[j];
    emit_node(codes + o, sorted + o, S.off[j + 1] - o, i - o, S.nodes[j], S.leaf_parent[j], S.perm[j], S.span[j]);
}

__device__ __forceinline__ float aload(const float* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Leaf slot l climbs from its box towards the root (the second arrival at a
// node merges both child boxes and goes on).  Nodes handed over between
// threads of different blocks use device-scope atomics and a device-scope
// acquire-release counter.
__device__ __forceinline__ bool climb_global(float (&lo)[3], float (&hi)[3], int idx, int side, BNode* nodes,
                                             uint32_t* counters) {
    float* nb = (float*)&nodes[idx];
    float* dst = nb + (side ? 6 : 0);
    for (int c = 0; c < 3; c++) {
        __hip_atomic_store(dst + c, lo[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(dst + 3 + c, hi[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // release our box, acquire the sibling's: the second arrival sees both
    uint32_t old = __hip_atomic_fetch_add(&counters[idx], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (old == 0u) return false;
    const float* o = nb + (side ? 0 : 6);
    for (int c = 0; c < 3; c++) {
        lo[c] = fminf(lo[c], aload(o + c));
        hi[c] = fmaxf(hi[c], aload(o + 3 + c));
    }
    return true;
}

__device__ __forceinline__ void refit_leaf(const float* box, const uint32_t* perm, int l, BNode* nodes,
                                           const int* leaf_parent, uint32_t* counters) {
    const float* p = box + 6 * (long long)perm[l];
    float lo[3] = {p[0], p[1], p[2]}, hi[3] = {p[3], p[4], p[5]};
    uint32_t par = (uint32_t)leaf_parent[l];
    while (true) {
        int idx = (int)(par & 0x7FFFFFFFu);
        if (!climb_global(lo, hi, idx, (int)(par >> 31), nodes, counters)) return;
        if (idx == 0) return;
        par = (uint32_t)__hip_atomic_load(&((int*)&nodes[idx].m)[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void __launch_bounds__(256) k_refit(const float* box, const uint32_t* perm, int n, BNode* nodes,
                                               const int* leaf_parent, uint32_t* counters) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n) refit_leaf(box, perm, l, nodes, leaf_parent, counters);
}

// LBVH refit in two tiers.  A block owns the leaf slots [b0, b0 + kRefitTile); an
// internal node whose leaf range lies inside them (a Karras node is one end of
// its own range, so its number lies inside too) is merged in LDS under a
// workgroup-scope counter, and only the nodes whose range leaves the block
// take the device-scope hand-over above.  Once a climb leaves its block every
// ancestor's range does too.
constexpr int kRefitTile = 1024;

__device__ __forceinline__ void refit_leaf_lbvh(const float* box, const uint32_t* perm, int l, int b0, int b1,
                                                BNode* nodes, const int* leaf_parent, const int* span,
                                                uint32_t* counters, uint32_t* lcnt, float (*lbox)[2][6]) {
    const float* p = box + 6 * (long long)perm[l];
    float lo[3] = {p[0], p[1], p[2]}, hi[3] = {p[3], p[4], p[5]};
    uint32_t par = (uint32_t)leaf_parent[l];
    bool local = true;
    while (true) {
        int idx = (int)(par & 0x7FFFFFFFu);
        int side = (int)(par >> 31);
        if (local) {
            int o = span[idx];
            local = (idx < o ? idx : o) >= b0 && (idx < o ? o : idx) < b1;
        }
        if (local) {
            float* dst = (float*)&nodes[idx] + (side ? 6 : 0);
            float* mine = lbox[idx - b0][side];
            for (int c = 0; c < 3; c++) {
                dst[c] = lo[c];
                dst[3 + c] = hi[c];
                mine[c] = lo[c];
                mine[3 + c] = hi[c];
            }
            uint32_t old = __hip_atomic_fetch_add(&lcnt[idx - b0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0u) return;
            const float* other = lbox[idx - b0][side ^ 1];
            for (int c = 0; c < 3; c++) {
                lo[c] = fminf(lo[c], other[c]);
                hi[c] = fmaxf(hi[c], other[3 + c]);
            }
        } else if (!climb_global(lo, hi, idx, side, nodes, counters)) {
            return;
        }
        if (idx == 0) return;
        par = (uint32_t)((const int*)&nodes[idx].m)[2];
    }
}

__global__ void __launch_bounds__(kRefitTile) k_refit_lbvh(const float* box, const uint32_t* perm, int n,
                                                           BNode* nodes, const int* leaf_parent, const int* span,
                                                           uint32_t* counters) {
    __shared__ uint32_t lcnt[kRefitTile];
    __shared__ float lbox[kRefitTile][2][6];
    lcnt[threadIdx.x] = 0u;
    __syncthreads();
    int b0 = blockIdx.x * kRefitTile;
    int b1 = b0 + kRefitTile < n ? b0 + kRefitTile : n;
    int l = b0 + (int)threadIdx.x;
    if (l < n) refit_leaf_lbvh(box, perm, l, b0, b1, nodes, leaf_parent, span, counters, lcnt, lbox);
}

// arrival counters of every tree of a batch to zero ([max(n - 1, 1)] each)
__global__ void __launch_bounds__(256) k_refit_clear(BuildSet S) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.off[S.nj]) return;
    int j = job_of(S, i);
    int li = i - S.off[j], n = S.off[j + 1] - S.off[j];
    if (li < (n > 1 ? n - 1 : 1)) S.counters[j][li] = 0u;
}

// Every tree of a batch; a block covers kRefitTile leaf slots of one tree
// (tree j's blocks start at blk[j]).
__global__ void __launch_bounds__(kRefitTile) k_refit_batch(BuildSet S, RefitBlocks B) {
    __shared__ uint32_t lcnt[kRefitTile];
    __shared__ float lbox[kRefitTile][2][6];
    lcnt[threadIdx.x] = 0u;
    __syncthreads();
    int j = 0;
    while (j + 1 < S.nj && (int)blockIdx.x >= B.blk[j + 1]) j++;
    int n = S.off[j + 1] - S.off[j];
    int b0 = ((int)blockIdx.x - B.blk[j]) * kRefitTile;
    int b1 = b0 + kRefitTile < n ? b0 + kRefitTile : n;
    int l = b0 + (int)threadIdx.x;
    if (l < n)
        refit_leaf_lbvh(S.box[j], S.perm[j], l, b0, b1, S.nodes[j], S.leaf_parent[j], S.span[j], S.counters[j], lcnt,
                        lbox);
}

__global__ void __launch_bounds__(256) k_sah(const BNode* nodes, int n_int, double* out) {
    __shared__ double sh[256];
    double s = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_int; i += gridDim.x * blockDim.x) {
        BNode nd = nodes[i];
        float ex = nd.a.w - nd.a.x, ey = nd.b.x - nd.a.y, ez = nd.b.y - nd.a.z;
        if (ex >= 0) s += 2.0 * ((double)ex * ey + (double)ey * ez + (double)ez * ex);
        ex = nd.c.y - nd.b.z; ey = nd.c.z - nd.b.w; ez = nd.c.w - nd.c.x;
        if (ex >= 0) s += 2.0 * ((double)ex * ey + (double)ey * ez + (double)ez * ex);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, sh[0]);
}

// ---- top-down binned SAH build (the static scene, once per scene) ----
// The same node format as the LBVH, so every query runs on either tree.  A
// level of the build is one launch with one block per node: centroid bounds,
// kSahBins bins per axis (counts and primitive boxes), the split of least
// A_L N_L + A_R N_R, a stable partition of the node's primitive indices, and
// the two children (a one-primitive child is a leaf).  Internal nodes are
// numbered in depth-first order (a node's left child follows it, its right
// child follows the left subtree), so a walk down the near side reads nearby
// nodes.  Boxes come from a refit at the end.  Where every centroid falls in
// one bin the range is cut in half.
constexpr int kSahBins = 32;
struct SahItem { int node, start, count, pad; };

__device__ __forceinline__ int sah_bin(float c, float lo, float scale) {
    int b = (int)((c - lo) * scale);
    return b < 0 ? 0 : (b >= kSahBins ? kSahBins - 1 : b);
}

__global__ void __launch_bounds__(256) k_sah_level(const float* box, const SahItem* items, const uint32_t* idx_in,
                                                   uint32_t* idx_out, BNode* nodes, int* leaf_parent, uint32_t* perm,
                                                   SahItem* next, uint32_t* ctr) {
#pragma clang fp contract(off)
    __shared__ uint32_t s_cb[6];                      // centroid bounds (ordered floats)
    __shared__ uint32_t s_cnt[3][kSahBins];
    __shared__ uint32_t s_bb[3][kSahBins][6];         // bin boxes (ordered floats)
    __shared__ float s_cost[3];
    __shared__ int s_split[3];
    __shared__ uint32_t s_scan[256];
    const SahItem it = items[blockIdx.x];
    const int tid = threadIdx.x;
    auto cen = [&](uint32_t p, int ax) { return 0.5f * (box[6 * (long long)p + ax] + box[6 * (long long)p + 3 + ax]); };
    if (tid < 3) { s_cb[tid] = 0xFFFFFFFFu; s_cb[3 + tid] = 0u; }
    for (int k = tid; k < 3 * kSahBins; k += 256) {
        (&s_cnt[0][0])[k] = 0u;
        for (int j = 0; j < 3; j++) { (&s_bb[0][0][0])[6 * k + j] = 0xFFFFFFFFu; (&s_bb[0][0][0])[6 * k + 3 + j] = 0u; }
    }
    __syncthreads();
    for (int i = tid; i < it.count; i += 256) {
        uint32_t p = idx_in[it.start + i];
        for (int ax = 0; ax < 3; ax++) {
            uint32_t o = f2ord(cen(p, ax));
            atomicMin(&s_cb[ax], o);
            atomicMax(&s_cb[3 + ax], o);
        }
    }
    __syncthreads();
    float clo[3], scale[3];
    for (int ax = 0; ax < 3; ax++) {
        clo[ax] = ord2f(s_cb[ax]);
        float ext = ord2f(s_cb[3 + ax]) - clo[ax];
        scale[ax] = ext > 0.0f ? (float)kSahBins / ext : 0.0f;
    }
    for (int i = tid; i < it.count; i += 256) {
        uint32_t p = idx_in[it.start + i];
        const float* b = box + 6 * (long long)p;
        for (int ax = 0; ax < 3; ax++) {
            int k = sah_bin(cen(p, ax), clo[ax], scale[ax]);
            atomicAdd(&s_cnt[ax][k], 1u);
            for (int j = 0; j < 3; j++) {
                atomicMin(&s_bb[ax][k][j], f2ord(b[j]));
                atomicMax(&s_bb[ax][k][3 + j], f2ord(b[3 + j]));
            }
        }
    }
    __syncthreads();
    if (tid < 3) {  // sweep of axis tid: cost of cutting after bin s
        const int ax = tid;
        float rl[3] = {INFINITY, INFINITY, INFINITY}, rh[3] = {-INFINITY, -INFINITY, -INFINITY};
        float right_area[kSahBins];
        uint32_t right_n[kSahBins];
        uint32_t n = 0;
        for (int k = kSahBins - 1; k >= 1; k--) {
            if (s_cnt[ax][k]) {
                for (int j = 0; j < 3; j++) {
                    rl[j] = fminf(rl[j], ord2f(s_bb[ax][k][j]));
                    rh[j] = fmaxf(rh[j], ord2f(s_bb[ax][k][3 + j]));
                }
            }
            n += s_cnt[ax][k];
            float ex = rh[0] - rl[0], ey = rh[1] - rl[1], ez = rh[2] - rl[2];
            right_area[k] = n ? 2.0f * (ex * ey + ey * ez + ez * ex) : 0.0f;
            right_n[k] = n;
        }
        float ll[3] = {INFINITY, INFINITY, INFINITY}, lh[3] = {-INFINITY, -INFINITY, -INFINITY};
        uint32_t nl = 0;
        float best = INFINITY;
        int bs = -1;
        for (int k = 0; k < kSahBins - 1; k++) {
            if (s_cnt[ax][k]) {
                for (int j = 0; j < 3; j++) {
                    ll[j] = fminf(ll[j], ord2f(s_bb[ax][k][j]));
                    lh[j] = fmaxf(lh[j], ord2f(s_bb[ax][k][3 + j]));
                }
            }
            nl += s_cnt[ax][k];
            if (nl == 0 || right_n[k + 1] == 0) continue;
            float ex = lh[0] - ll[0], ey = lh[1] - ll[1], ez = lh[2] - ll[2];
            float cost = 2.0f * (ex * ey + ey * ez + ez * ex) * (float)nl + right_area[k + 1] * (float)right_n[k + 1];
            if (cost < best) { best = cost; bs = k; }
        }
        s_cost[ax] = best;
        s_split[ax] = bs;
    }
    __syncthreads();
    int axis = 0;
    for (int ax = 1; ax < 3; ax++)
        if (s_cost[ax] < s_cost[axis]) axis = ax;
    int split = s_split[axis];  // -1: cut the range in half
    const int half = it.count / 2;
    // count the left side with the same test the partition uses
    if (tid == 0) s_cb[0] = 0u;
    __syncthreads();
    if (split >= 0) {
        uint32_t mine = 0;
        for (int i = tid; i < it.count; i += 256)
            mine += sah_bin(cen(idx_in[it.start + i], axis), clo[axis], scale[axis]) <= split ? 1u : 0u;
        atomicAdd(&s_cb[0], mine);
    }
    __syncthreads();
    uint32_t n_left = split >= 0 ? s_cb[0] : (uint32_t)half;
    if (n_left == 0u || n_left >= (uint32_t)it.count) {
        split = -1;
        n_left = (uint32_t)half;
    }
    // stable partition, 256 indices at a time
    uint32_t base_l = 0, base_r = 0;
    for (int c0 = 0; c0 < it.count; c0 += 256) {
        const int i = c0 + tid;
        const bool act = i < it.count;
        uint32_t p = act ? idx_in[it.start + i] : 0u;
        bool left = false;
        if (act) left = split >= 0 ? sah_bin(cen(p, axis), clo[axis], scale[axis]) <= split : i < half;
        s_scan[tid] = left ? 1u : 0u;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {  // inclusive scan
            uint32_t y = tid >= o ? s_scan[tid - o] : 0u;
            __syncthreads();
            s_scan[tid] += y;
            __syncthreads();
        }
        const uint32_t incl = s_scan[tid];
        const uint32_t tot_l = s_scan[255];
        const int n_act = min(256, it.count - c0);
        if (act) {
            uint32_t dst = left ? base_l + incl - 1u : n_left + base_r + ((uint32_t)tid + 1u - incl) - 1u;
            idx_out[it.start + dst] = p;
        }
        base_l += tot_l;
        base_r += (uint32_t)n_act - tot_l;
        __syncthreads();
    }
    if (tid < 2) {
        const int side = tid;
        const int cs = side ? it.start + (int)n_left : it.start;
        const int cn = side ? it.count - (int)n_left : (int)n_left;
        int child;
        if (cn == 1) {
            child = (int)(EMRT_LEAF | (uint32_t)cs);
            perm[cs] = idx_out[cs];
            leaf_parent[cs] = (int)((uint32_t)it.node | (side ? EMRT_SIDE : 0u));
        } else {
            // depth-first order: the left subtree's n_left - 1 internal nodes follow the node
            child = side ? it.node + (int)n_left : it.node + 1;
            ((int*)&nodes[child].m)[2] = (int)((uint32_t)it.node | (side ? EMRT_SIDE : 0u));
            uint32_t q = atomicAdd(&ctr[0], 1u);
            next[q] = SahItem{child, cs, cn, 0};
        }
        int* m = (int*)&nodes[it.node].m;
        m[side] = child;
        if (side == 0) m[3] = axis;
    }
}

__global__ void k_sah_init(uint32_t* idx, int n, SahItem* items, BNode* nodes, uint32_t* ctr) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) idx[i] = (uint32_t)i;
    if (i == 0) {
        items[0] = SahItem{0, 0, n, 0};
        ((int*)&nodes[0].m)[2] = -1;
        ctr[0] = 0u;  // items of the next level
    }
}

int bvh_build_sah(const float* box6, int n, Tree& tree, const BuildTemp& tmp, hipStream_t st) {
    if (n < 2) {
        bvh_build(box6, n, tree, tmp, st);
        return 0;
    }
    tree.n = n;
    tree.lbvh = false;
    SahItem* items[2] = {(SahItem*)tmp.k0, (SahItem*)tmp.k1};  // each holds cap / 2 items >= n / 2
    uint32_t* idx[2] = {tmp.v0, tmp.v1};
    uint32_t* ctr = tmp.bounds;
    hipLaunchKernelGGL(k_sah_init, dim3((n + 255) / 256), dim3(256), 0, st, idx[0], n, items[0], tree.nodes, ctr);
    int n_items = 1, cur = 0, levels = 0;
    while (n_items > 0) {
        hipLaunchKernelGGL(k_fill_zero1, dim3(1), dim3(1), 0, st, ctr);
        hipLaunchKernelGGL(k_sah_level, dim3(n_items), dim3(256), 0, st, box6, items[cur], idx[cur], idx[1 - cur],
                           tree.nodes, tree.leaf_parent, tree.perm, items[1 - cur], ctr);
        uint32_t h = 0;
        if (hipMemcpyAsync(&h, ctr, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
        if (hipStreamSynchronize(st) != hipSuccess) return -1;
        n_items = (int)h;
        cur = 1 - cur;
        if (++levels > n) return -1;  // a level always splits every range: cannot happen
    }
    bvh_refit(box6, tree, st);
    return levels;
}

size_t build_temp_bytes(long long cap) {
    if (cap < 1) cap = 1;
    size_t b = 0;
    b += 2 * sizeof(unsigned long long) * (size_t)cap;
    b += 2 * sizeof(uint32_t) * (size_t)cap;
    b += 256;
    b += radix_temp_bytes(cap);
    return b + 5 * 256;
}

static char* align256(char* p) { return (char*)(((uintptr_t)p + 255) & ~(uintptr_t)255); }

void carve_build_temp(void* base, long long cap, BuildTemp& t) {
    if (cap < 1) cap = 1;
    char* p = align256((char*)base);
    t.k0 = (unsigned long long*)p; p = align256(p + sizeof(unsigned long long) * cap);
    t.k1 = (unsigned long long*)p; p = align256(p + sizeof(unsigned long long) * cap);
    t.v0 = (uint32_t*)p; p = align256(p + sizeof(uint32_t) * cap);
    t.v1 = (uint32_t*)p; p = align256(p + sizeof(uint32_t) * cap);
    t.bounds = (uint32_t*)p; p = align256(p + 256);
    t.radix = p;
}

// Morton bits per axis for trees of up to n primitives: about 2^12 cells or
// more per primitive, at least 10 bits (a 32-bit sort key for four trees).
static int morton_bits(int n) {
    int lg = 0;
    while (lg < 31 && (1LL << lg) < (long long)n) lg++;
    int b = (lg + 2) / 3 + 4;
    return b < 10 ? 10 : (b > 20 ? 20 : b);
}

void bvh_build_many(const BuildJob* jobs, int n_jobs, const BuildTemp& tmp, hipStream_t st) {
    BuildSet S{};
    int total = 0, n_max = 0;
    for (int k = 0; k < n_jobs; k++) {
        jobs[k].tree->n = jobs[k].n > 0 ? jobs[k].n : 0;
        if (jobs[k].n <= 0) continue;
        int j = S.nj++;
        Tree& t = *jobs[k].tree;
        S.box[j] = jobs[k].box6;
        S.nodes[j] = t.nodes;
        S.leaf_parent[j] = t.leaf_parent;
        S.perm[j] = t.perm;
        S.counters[j] = t.counters;
        S.span[j] = t.span;
        t.lbvh = true;
        S.off[j] = total;
        total += jobs[k].n;
        n_max = jobs[k].n > n_max ? jobs[k].n : n_max;
    }
    S.off[S.nj] = total;
    if (total == 0) return;
    S.bits = morton_bits(n_max);
    int job_bits = S.nj > 2 ? 2 : (S.nj > 1 ? 1 : 0);
    int g = (total + 255) / 256;
    hipLaunchKernelGGL(k_init_bounds, dim3(1), dim3(64), 0, st, tmp.bounds, S.nj);
    hipLaunchKernelGGL(k_bounds, dim3(g), dim3(256), 0, st, S, tmp.bounds);
    hipLaunchKernelGGL(k_morton, dim3(g), dim3(256), 0, st, S, tmp.bounds, tmp.k0, tmp.v0);
    int which = radix_sort(tmp.k0, tmp.v0, tmp.k1, tmp.v1, nullptr, total, 3 * S.bits + job_bits, tmp.radix, st);
    hipLaunchKernelGGL(k_emit, dim3(g), dim3(256), 0, st, S, which ? tmp.k1 : tmp.k0, which ? tmp.v1 : tmp.v0);
    RefitBlocks B{};
    for (int j = 0; j < S.nj; j++) B.blk[j + 1] = B.blk[j] + (S.off[j + 1] - S.off[j] + kRefitTile - 1) / kRefitTile;
    hipLaunchKernelGGL(k_refit_clear, dim3(g), dim3(256), 0, st, S);
    hipLaunchKernelGGL(k_refit_batch, dim3(B.blk[S.nj]), dim3(kRefitTile), 0, st, S, B);
}

void bvh_build(const float* box6, int n, Tree& tree, const BuildTemp& tmp, hipStream_t st) {
    BuildJob job{box6, n, &tree};
    bvh_build_many(&job, 1, tmp, st);
}

// Tree quality for the rebuild-on-degradation policy: out[0] = the summed
// surface area of every node's two child boxes, out[1] = the root box's
// (their ratio is the expected number of box tests of a random ray).
__device__ __forceinline__ double half_area(float lx, float ly, float lz, float hx, float hy, float hz) {
    const double x = fmax((double)hx - lx, 0.0), y = fmax((double)hy - ly, 0.0), z = fmax((double)hz - lz, 0.0);
    return x * y + y * z + z * x;
}

__global__ void __launch_bounds__(256) k_tree_quality(const BNode* nodes, int n_int, double* out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_int; i += gridDim.x * blockDim.x) {
        const BNode nd = nodes[i];
        s += half_area(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y) +
             half_area(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&out[0], sh[0]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const BNode r = nodes[0];
        out[1] = half_area(fminf(r.a.x, r.b.z), fminf(r.a.y, r.b.w), fminf(r.a.z, r.c.x), fmaxf(r.a.w, r.c.y),
                           fmaxf(r.b.x, r.c.z), fmaxf(r.b.y, r.c.w));
    }
}

void tree_quality(const Tree& tree, double* out2, hipStream_t st) {
    fill_u64((unsigned long long*)out2, 0ULL, 2, st);
    const int n_int = tree.n - 1;
    if (n_int < 1) return;
    const int g = std::min((n_int + 255) / 256, 64);
    hipLaunchKernelGGL(k_tree_quality, dim3(g), dim3(256), 0, st, tree.nodes, n_int, out2);
}

void bvh_refit(const float* box6, Tree& tree, hipStream_t st) {
    int n = tree.n;
    if (n <= 0) return;
    fill_u32(tree.counters, 0u, n > 1 ? n - 1 : 1, st);
    if (tree.lbvh)
        hipLaunchKernelGGL(k_refit_lbvh, dim3((n + kRefitTile - 1) / kRefitTile), dim3(kRefitTile), 0, st, box6,
                           tree.perm, n, tree.nodes, tree.leaf_parent, tree.span, tree.counters);
    else
        hipLaunchKernelGGL(k_refit, dim3((n + 255) / 256), dim3(256), 0, st, box6, tree.perm, n, tree.nodes,
                           tree.leaf_parent, tree.counters);
}

void bvh_sah(const Tree& tree, double* out, hipStream_t st) {
    int n_int = tree.n > 1 ? tree.n - 1 : 1;
    if (tree.n <= 0) return;
    int g = (n_int + 255) / 256;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_sah, dim3(g), dim3(256), 0, st, tree.nodes, n_int, out);
}


// ------------------------------------------------------ 4-wide tree ----
// Host-side collapse of a binary tree into 4-wide nodes: a node takes its
// binary node's two children and keeps opening the internal child of
// largest surface area until it has four (or only leaves).  Child boxes are
// quantised to bytes on a per-node grid o + q 2^e: the low byte is the
// largest q whose fused multiply-add fma(q, 2^e, o) lies at or below the
// child's low bound, the high byte the smallest at or above its high bound,
// evaluated with the same fma the traversal uses, so the decoded boxes
// contain the children's boxes exactly.  A node's children get consecutive
// indices, before the subtrees below them.  The nodes of the top
// kBvh4TopLevels levels are numbered breadth first (so the tree's top is an
// index prefix, which the traversal keeps in LDS), the rest depth first.
namespace {
struct HBox {
    float lo[3], hi[3];
};

HBox child_box(const BNode& n, int side) {
    HBox b;
    if (side == 0) {
        b.lo[0] = n.a.x; b.lo[1] = n.a.y; b.lo[2] = n.a.z;
        b.hi[0] = n.a.w; b.hi[1] = n.b.x; b.hi[2] = n.b.y;
    } else {
        b.lo[0] = n.b.z; b.lo[1] = n.b.w; b.lo[2] = n.c.x;
        b.hi[0] = n.c.y; b.hi[1] = n.c.z; b.hi[2] = n.c.w;
    }
    return b;
}

bool box_empty(const HBox& b) {
    for (int k = 0; k < 3; k++)
        if (!(b.lo[k] <= b.hi[k])) return true;
    return false;
}

double box_area(const HBox& b) {
    const double x = (double)b.hi[0] - b.lo[0], y = (double)b.hi[1] - b.lo[1], z = (double)b.hi[2] - b.lo[2];
    return x * y + y * z + z * x;
}

float scale_of(uint32_t e) {
    const uint32_t bits = e << 23;
    float f;
    memcpy(&f, &bits, sizeof(f));
    return f;
}

// exponent byte e of the grid step 2^(e - 127) so that fma(255, step, o) >= hi
// (0, a step of 0, when the node is flat on this axis)
uint32_t grid_exp(float o, float hi) {
    if (!(hi > o)) return 0;
    int e2 = 0;
    frexp(((double)hi - (double)o) / 255.0, &e2);
    int e = e2 + 127;
    if (e < 1) e = 1;
    while (e < 254 && fmaf(255.0f, scale_of((uint32_t)e), o) < hi) e++;
    return (uint32_t)e;
}

uint32_t q_low(float v, float o, float step) {
    if (step == 0.0f) return 0u;
    double q = floor(((double)v - (double)o) / (double)step);
    q = q < 0.0 ? 0.0 : (q > 255.0 ? 255.0 : q);
    uint32_t k = (uint32_t)q;
    while (k > 0 && fmaf((float)k, step, o) > v) k--;
    while (k < 255 && fmaf((float)(k + 1), step, o) <= v) k++;
    return k;
}

uint32_t q_high(float v, float o, float step) {
    if (step == 0.0f) return 0u;
    double q = ceil(((double)v - (double)o) / (double)step);
    q = q < 0.0 ? 0.0 : (q > 255.0 ? 255.0 : q);
    uint32_t k = (uint32_t)q;
    while (k < 255 && fmaf((float)k, step, o) < v) k++;
    while (k > 0 && fmaf((float)(k - 1), step, o) >= v) k--;
    return k;
}

struct Ent {
    int ref;  // internal binary node index, or EMRT_LEAF | primitive slot (negative)
    HBox box;
};
}  // namespace

int bvh4_collapse(const BNode* bin, int n_prims, QNode4* out, int cap) {
    if (n_prims <= 0 || cap < 1) return 0;
    struct Work {
        int nid, slot, depth;  // binary node, 4-wide slot, depth of the 4-wide node
    };
    std::deque<Work> work;
    int n_out = 1;
    work.push_back({0, 0, 0});
    while (!work.empty()) {
        // breadth first while the oldest entry is above the staged depth
        // (then every entry left is at that depth), depth first below
        const bool bfs = work.front().depth < kBvh4TopLevels;
        const Work w = bfs ? work.front() : work.back();
        if (bfs) work.pop_front();
        else work.pop_back();
        const int nid = w.nid, oi = w.slot;
        Ent ch[4];
        int n = 0;
        for (int side = 0; side < 2; side++) {
            const HBox b = child_box(bin[nid], side);
            if (!box_empty(b)) ch[n++] = Ent{side ? bin[nid].m.y : bin[nid].m.x, b};
        }
        while (n < 4) {  // open the internal child of largest area
            int best = -1;
            double ba = -1.0;
            for (int k = 0; k < n; k++)
                if (ch[k].ref >= 0 && box_area(ch[k].box) > ba) { ba = box_area(ch[k].box); best = k; }
            if (best < 0) break;
            const BNode& cn = bin[ch[best].ref];
            Ent e[2];
            int ne = 0;
            for (int side = 0; side < 2; side++) {
                const HBox b = child_box(cn, side);
                if (!box_empty(b)) e[ne++] = Ent{side ? cn.m.y : cn.m.x, b};
            }
            if (ne == 0) { ch[best] = ch[--n]; continue; }
            ch[best] = e[0];
            if (ne == 2) ch[n++] = e[1];
        }
        QNode4 q{};
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int k = 0; k < n; k++)
            for (int a = 0; a < 3; a++) {
                lo[a] = fminf(lo[a], ch[k].box.lo[a]);
                hi[a] = fmaxf(hi[a], ch[k].box.hi[a]);
            }
        if (n == 0)
            for (int a = 0; a < 3; a++) lo[a] = hi[a] = 0.0f;
        uint32_t e[3], qx[3] = {0, 0, 0}, rx[3] = {0, 0, 0};
        for (int a = 0; a < 3; a++) e[a] = grid_exp(lo[a], hi[a]);
        int c[4] = {0, 0, 0, 0};
        for (int k = 0; k < n; k++) {
            for (int a = 0; a < 3; a++) {
                const float step = e[a] ? scale_of(e[a]) : 0.0f;
                qx[a] |= q_low(ch[k].box.lo[a], lo[a], step) << (8 * k);
                rx[a] |= q_high(ch[k].box.hi[a], lo[a], step) << (8 * k);
            }
            if (ch[k].ref >= 0) {  // an internal child becomes the next 4-wide slot
                if (n_out >= cap) return -1;
                c[k] = n_out;
                work.push_back({ch[k].ref, n_out++, w.depth + 1});
            } else {
                c[k] = ch[k].ref;
            }
        }
        const uint32_t meta = e[0] | (e[1] << 8) | (e[2] << 16) | ((uint32_t)n << 24);
        float mw;
        memcpy(&mw, &meta, sizeof(mw));
        q.o = make_float4(lo[0], lo[1], lo[2], mw);
        q.q = make_uint4(qx[0], qx[1], qx[2], 0u);
        q.r = make_uint4(rx[0], rx[1], rx[2], 0u);
        q.c = make_int4(c[0], c[1], c[2], c[3]);
        out[oi] = q;
    }
    return n_out;
}

}  // namespace emrt
