// trace.hip -- shooting and bouncing rays from the transmitters.
//
// Section II-A: the engine traces direct, reflected and diffracted rays
// through a BVH and caches the propagation paths it finds.  Here each
// transmitter launches N rays on a Fibonacci sphere; every bounce is one
// launch of k_bounce, a persistent kernel whose waves pull 64-ray chunks
// from a device counter.  Per ray and bounce it
//   1. finds the closest hit in the static tree (4-wide, quantised boxes) and
//      the dynamic LBVH (short stack, nearer child first, watertight triangle
//      test, previous face excluded, ties to the lowest triangle id),
//   2. records the hit triangle in the per-bounce hit log,
//   3. captures receivers whose reception sphere (radius k alpha (L + s),
//      alpha = sqrt(4 pi / N)) the segment crosses, inserting the path key
//      (tx, rx, face sequence) into the lock-free path table,
//   4. on the first segment, marks wedge edges that the ray passes within
//      k alpha s of (diffraction candidates),
//   5. reflects specularly and appends the surviving ray to the next
//      bounce's buffer with one atomic per wave (ballot + mbcnt prefix).
#include <algorithm>

#include "emrt_dev.h"
#include "emrt_launch.h"

namespace emrt {

__device__ __forceinline__ void fib_dir(long long i, int N, float& x, float& y, float& z) {
    const double ga = kPi * (3.0 - sqrt(5.0));
    double zz = 1.0 - (2.0 * (double)i + 1.0) / (double)N;
    double r = sqrt(1.0 - zz * zz);
    double ph = (double)i * ga;
    double s, c;
    sincos(ph, &s, &c);
    x = (float)(r * c);
    y = (float)(r * s);
    z = (float)zz;
}

// Morton code of each launch direction, so that neighbouring threads trace
// neighbouring directions (the launch index still identifies the ray).
__global__ void k_dir_codes(int N, unsigned long long* codes, uint32_t* vals) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float x, y, z;
    fib_dir(i, N, x, y, z);
    auto q = [](float v) { return (uint32_t)(fminf(fmaxf(0.5f * (v + 1.0f), 0.0f), 1.0f) * 2097151.0f); };
    auto split3 = [](uint32_t a) {
        unsigned long long x = a & 0x1fffffu;
        x = (x | x << 32) & 0x1f00000000ffffULL;
        x = (x | x << 16) & 0x1f0000ff0000ffULL;
        x = (x | x << 8) & 0x100f00f00f00f00fULL;
        x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
        x = (x | x << 2) & 0x1249249249249249ULL;
        return x;
    };
    codes[i] = (split3(q(x)) << 2) | (split3(q(y)) << 1) | split3(q(z));
    vals[i] = (uint32_t)i;
}

__global__ void k_copy_perm(const uint32_t* in, uint32_t* out, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

void ray_order(int N, uint32_t* perm, const BuildTemp& tmp, hipStream_t st) {
    int g = (N + 255) / 256;
    hipLaunchKernelGGL(k_dir_codes, dim3(g), dim3(256), 0, st, N, tmp.k0, tmp.v0);
    int which = radix_sort(tmp.k0, tmp.v0, tmp.k1, tmp.v1, nullptr, N, 63, tmp.radix, st);
    hipLaunchKernelGGL(k_copy_perm, dim3(g), dim3(256), 0, st, which ? tmp.v1 : tmp.v0, perm, N);
}

__global__ void __launch_bounds__(256) k_raygen(const double* tx_pos, int n_tx, int N, const uint32_t* perm,
                                                RaySoA out, unsigned long long* n_out) {
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long total = (long long)n_tx * N;
    if (k == 0) *n_out = (unsigned long long)total;
    if (k >= total) return;
    int tx = (int)(k / N);
    int t = (int)(k - (long long)tx * N);
    uint32_t i = perm ? perm[t] : (uint32_t)t;
    float x, y, z;
    fib_dir(i, N, x, y, z);
    out.ox[k] = (float)tx_pos[3 * tx];
    out.oy[k] = (float)tx_pos[3 * tx + 1];
    out.oz[k] = (float)tx_pos[3 * tx + 2];
    out.dx[k] = x;
    out.dy[k] = y;
    out.dz[k] = z;
    out.L[k] = 0.0f;
    out.id[k] = (uint32_t)k;  // the launch slot: the hit log rows are then written in launch order
    out.prev[k] = -1;
}

__global__ void k_dir_table(const uint32_t* perm, int N, float4* dirs) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    float x, y, z;
    fib_dir(perm[t], N, x, y, z);
    dirs[t] = make_float4(x, y, z, 0.0f);
}

void dir_table(const uint32_t* perm, int N, float4* dirs, hipStream_t st) {
    if (N > 0) hipLaunchKernelGGL(k_dir_table, dim3((N + 255) / 256), dim3(256), 0, st, perm, N, dirs);
}

void raygen(const double* tx_pos, int n_tx, int N, const uint32_t* perm, RaySoA out, unsigned long long* n_out,
            hipStream_t st) {
    long long total = (long long)n_tx * N;
    long long g = (total + 255) / 256;
    hipLaunchKernelGGL(k_raygen, dim3((unsigned)(g < 1 ? 1 : g)), dim3(256), 0, st, tx_pos, n_tx, N, perm, out, n_out);
}

// far bound of the distance from o to any point of a tree's root box
__device__ __forceinline__ float root_far(const Bvh& t, float ox, float oy, float oz) {
    BNode nd = t.nodes[0];
    float lx = fminf(nd.a.x, nd.b.z), ly = fminf(nd.a.y, nd.b.w), lz = fminf(nd.a.z, nd.c.x);
    float hx = fmaxf(nd.a.w, nd.c.y), hy = fmaxf(nd.b.x, nd.c.z), hz = fmaxf(nd.b.y, nd.c.w);
    float dx = fmaxf(fabsf(lx - ox), fabsf(hx - ox));
    float dy = fmaxf(fabsf(ly - oy), fabsf(hy - oy));
    float dz = fmaxf(fabsf(lz - oz), fabsf(hz - oz));
    return sqrtf(dx * dx + dy * dy + dz * dz) * 1.0001f + 1.0f;
}

// Regroup key of a ray (BounceArgs::out_key): Morton order of its origin's
// cell on a 16 x 16 grid, then the octant of its direction.
__device__ __forceinline__ uint16_t regroup_key(const BounceArgs& a, float ox, float oy, float dx, float dy, float dz) {
    const float fx = (ox - a.key_ox) * a.key_sx, fy = (oy - a.key_oy) * a.key_sy;
    const uint32_t cx = fx > 0.0f ? (fx < 15.0f ? (uint32_t)fx : 15u) : 0u;
    const uint32_t cy = fy > 0.0f ? (fy < 15.0f ? (uint32_t)fy : 15u) : 0u;
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) m |= ((cx >> k) & 1u) << (2 * k) | ((cy >> k) & 1u) << (2 * k + 1);
    const uint32_t oct = (dx < 0.0f ? 1u : 0u) | (dy < 0.0f ? 2u : 0u) | (dz < 0.0f ? 4u : 0u);
    return (uint16_t)((m << 3) | oct);
}

// capture of a marked ray into the debug log
__device__ __forceinline__ void debug_log(const BounceArgs& a, uint32_t id, int b, int kind, int target) {
    if (!((a.dbg_sel[id >> 5] >> (id & 31)) & 1u)) return;
    const unsigned long long k = atomicAdd(a.dbg_n, 1ULL);
    if (k >= (unsigned long long)a.dbg_cap) return;
    a.dbg_log[3 * k] = (int)id;
    a.dbg_log[3 * k + 1] = b | (kind << 8);
    a.dbg_log[3 * k + 2] = target;
}

// One 64-ray chunk of a bounce: rays [base, base + 64) of the live buffer.
// REV: a launch from receivers (a.src.src_rx) whose spheres sit on the
// transmitters; the captured key is reversed into transmitter-to-receiver
// order (expand_ref rebuilds the same key from the reference).
template <bool STATS, bool REV>
__device__ __forceinline__ void bounce_chunk(const BounceArgs& a, unsigned long long n_in, unsigned long long base,
                                             int lane, unsigned& s_nodes, unsigned& s_tris, unsigned& s_seg,
                                             unsigned& s_cap, unsigned& s_box4, LdsStack* stk, int width = 64,
                                             const QNode4* top = nullptr, int n_top = 0) {
    const int b = a.b;
    unsigned long long i = base + (unsigned long long)lane;
    bool act = lane < width && i < n_in;
    float ox = 0, oy = 0, oz = 0, dx = 0, dy = 0, dz = 1, L = 0;
    uint32_t id = 0;
    int prev = -1;
    if (act && a.gen_dirs) {  // primary ray: the same values k_raygen would store
        const long long src = (long long)(i / (unsigned long long)a.gen_N);
        const float4 d = a.gen_dirs[i - (unsigned long long)src * (unsigned long long)a.gen_N];
        ox = (float)a.gen_src[3 * src]; oy = (float)a.gen_src[3 * src + 1]; oz = (float)a.gen_src[3 * src + 2];
        dx = d.x; dy = d.y; dz = d.z;
        id = (uint32_t)i;
    } else if (act) {
        ox = a.in.ox[i]; oy = a.in.oy[i]; oz = a.in.oz[i];
        dx = a.in.dx[i]; dy = a.in.dy[i]; dz = a.in.dz[i];
        L = a.in.L[i];
        id = a.in.id[i];
        prev = a.in.prev[i];
    }
    RayPre r = ray_pre(ox, oy, oz, dx, dy, dz);
    float best_t = INFINITY;
    int best_tri = 0x7FFFFFFF, best_face = -1;
    if (act) {
        if (STATS) s_seg++;
        closest_hit4<STATS>(a.st4, a.st, a.st_prims, r, prev, best_t, best_tri, best_face, s_box4, s_nodes, s_tris,
                            stk, top, n_top);
        closest_hit<STATS>(a.dy, a.dy_prims, r, prev, best_t, best_tri, best_face, s_nodes, s_tris, stk);
    }
    bool hit = act && best_tri != 0x7FFFFFFF;
    if (act) a.hitlog[(long long)b * a.n_total + id] = hit ? best_tri : -1;
    float t_end = hit ? best_t : INFINITY;

    // receiver capture on segments after at least one reflection
    if (act && b >= 1 && a.rxt.n_prims > 0) {
        float tcap = fminf(t_end, root_far(a.rxt, ox, oy, oz));
        float grow = a.alpha_k * (L + tcap);
        KeyRec mine;
        bool have = false;
        uint64_t h = 0;
        all_hits(a.rxt, r, tcap, grow, [&](int slot) {
            float4 p = a.rx_prims[slot];
            float wx = p.x - ox, wy = p.y - oy, wz = p.z - oz;
            float s = wx * dx + wy * dy + wz * dz;
            if (!(s > 0.0f && s < t_end)) return;
            float rho2 = wx * wx + wy * wy + wz * wz - s * s;
            float rs = a.alpha_k * (L + s);
            if (!(rho2 < rs * rs)) return;
            int target = __float_as_int(p.w);
            if (!REV && a.dbg_sel) debug_log(a, id, b, 0, target);
            if (!have) {
                const int source = (int)(id / (uint32_t)a.rays_per_tx);
                mine.to = KT_SPEC | (b << 8);
                if (REV) {
                    mine.rx = a.src.src_rx[source];
                    for (int j = 0; j < 5; j++)
                        mine.ids[j] = j < b ? a.src.tri_face[a.hitlog[(long long)(b - 1 - j) * a.n_total + id]] : -1;
                } else {
                    mine.tx = source;
                    for (int j = 0; j < 5; j++)
                        mine.ids[j] = j < b ? a.src.tri_face[a.hitlog[(long long)j * a.n_total + id]] : -1;
                }
                have = true;
            }
            if (REV) mine.tx = target;
            else mine.rx = target;
            h = key_hash(mine.tx, mine.rx, mine.to, mine.ids);
            int res = table_insert<REV ? 1 : 0>(a.table, a.mask, ref_ray(b, target, id), mine, h, a.src);
            if (res < 0) atomicOr(a.flags, FLAG_TABLE_FULL);
            if (STATS) s_cap++;
        }, stk);
    }

    // edge capture on the first segment (and, for reflection-diffraction
    // paths, on the second): radius k_rx alpha (L + s) as for receivers.  The
    // edges of static objects and of moving ones sit in two trees.
    if (act && (b == 0 || (b == 1 && a.diffraction == 2)) && a.diffraction &&
        (a.ets.n_prims > 0 || a.etd.n_prims > 0)) {
        const int source = (int)(id / (uint32_t)a.rays_per_tx);  // row of the illumination bitmap
        const int face1 = b == 1 ? a.src.tri_face[a.hitlog[id]] : -1;  // face of the first reflection
        auto edge_leaf = [&](const float4* prims, int slot) {
            float4 P0 = prims[2 * slot], P1 = prims[2 * slot + 1];
            float ex = P1.x - P0.x, ey = P1.y - P0.y, ez = P1.z - P0.z;
            float wx = ox - P0.x, wy = oy - P0.y, wz = oz - P0.z;
            float aa = dx * dx + dy * dy + dz * dz;
            float bb = dx * ex + dy * ey + dz * ez;
            float cc = ex * ex + ey * ey + ez * ez;
            float dd = dx * wx + dy * wy + dz * wz;
            float ee = ex * wx + ey * wy + ez * wz;
            float den = aa * cc - bb * bb;
            if (!(den > 1e-12f * aa * cc)) return;
            float s = (bb * ee - cc * dd) / den;
            float u = (aa * ee - bb * dd) / den;
            if (!(s > 0.0f && s < t_end && u > 0.0f && u < 1.0f)) return;
            float qx = ox + s * dx - (P0.x + u * ex);
            float qy = oy + s * dy - (P0.y + u * ey);
            float qz = oz + s * dz - (P0.z + u * ez);
            float re = a.alpha_k * (L + s);
            if (!(qx * qx + qy * qy + qz * qz < re * re)) return;
            int e = __float_as_int(P0.w);
            if (!REV && a.dbg_sel) debug_log(a, id, b, 1, e);
            if (b == 0) {
                uint32_t* w = a.illum + (long long)source * a.e_words + (e >> 5);
                uint32_t bit = 1u << (e & 31);
                if (!(__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit)) atomicOr(w, bit);
            } else if (!pair_insert(a.pairs, a.pair_mask, pair_key(source, face1, e))) {
                atomicOr(a.flags, FLAG_CAND_CAP);
            }
        };
        if (a.ets.n_prims > 0) {
            const float tcap = fminf(t_end, root_far(a.ets, ox, oy, oz));
            all_hits(a.ets, r, tcap, a.alpha_k * (L + tcap), [&](int slot) { edge_leaf(a.eprims_s, slot); }, stk);
        }
        if (a.etd.n_prims > 0) {
            const float tcap = fminf(t_end, root_far(a.etd, ox, oy, oz));
            all_hits(a.etd, r, tcap, a.alpha_k * (L + tcap), [&](int slot) { edge_leaf(a.eprims_d, slot); }, stk);
        }
    }

    // specular reflection about the face plane
    bool alive = hit && b < a.K;
    if (act && !alive) a.depth[id] = (uint8_t)b;
    float nox = 0, noy = 0, noz = 0, ndx = 0, ndy = 0, ndz = 0;
    if (alive) {
        const double* pl = a.plane + 4 * (long long)best_face;
        float nx = (float)pl[0], ny = (float)pl[1], nzv = (float)pl[2];
        nox = ox + best_t * dx;
        noy = oy + best_t * dy;
        noz = oz + best_t * dz;
        float dn = 2.0f * (dx * nx + dy * ny + dz * nzv);
        ndx = dx - dn * nx;
        ndy = dy - dn * ny;
        ndz = dz - dn * nzv;
    }
    long long o = wave_append(a.n_out, alive);
    if (alive) {
        a.out.ox[o] = nox; a.out.oy[o] = noy; a.out.oz[o] = noz;
        a.out.dx[o] = ndx; a.out.dy[o] = ndy; a.out.dz[o] = ndz;
        a.out.L[o] = L + best_t;
        a.out.id[o] = id;
        a.out.prev[o] = best_face;
        if (a.out_key) a.out_key[o] = regroup_key(a, nox, noy, ndx, ndy, ndz);
    }
}

template <bool STATS>
__device__ __forceinline__ void flush_stats(unsigned long long* stats, int lane, unsigned s_nodes, unsigned s_tris,
                                            unsigned s_seg, unsigned s_cap, unsigned s_box4) {
    if (STATS) {
        // [0] binary node visits, [1] triangle tests, [2] segments, [3] captures, [16] 4-wide child boxes tested
        unsigned long long v[5] = {s_nodes, s_tris, s_seg, s_cap, s_box4};
        const int slot[5] = {0, 1, 2, 3, 16};
        for (int k = 0; k < 5; k++) {
            unsigned long long x = v[k];
            for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off);
            if (lane == 0 && x) atomicAdd(&stats[slot[k]], x);
        }
    }
}

// Persistent: waves pull chunks of rays from a device counter and trace them
// 64 at a time; the traversal stacks live in LDS (one column per thread).
// Bounces 0 and 1 take 128 rays per chunk: their rays are still coherent, so
// the second 64 find the nodes the first brought into the CU's cache.  From
// bounce 2 on the rays are scattered and 64-ray chunks balance the tail
// better (measured: 6.10-6.17 against 6.33 ms of bounces per city frame).
#ifndef EMRT_BOUNCE_CHUNK
#define EMRT_BOUNCE_CHUNK 128
#endif
constexpr int kBounceChunk = EMRT_BOUNCE_CHUNK;  // rays per fetch, bounces 0 and 1 (a multiple of 64)
constexpr int kBounceChunkLate = 64;              // rays per fetch from bounce 2 on

template <bool STATS, bool REV>
__global__ void __launch_bounds__(256) k_bounce(BounceArgs a) {
    __shared__ int stk_lds[kStackRows][kStackStride];
    __shared__ QNode4 top[kTop4 > 0 ? kTop4 : 1];
    LdsStack stk{&stk_lds[0][threadIdx.x]};
    const int lane = lane_id();
    const unsigned long long n_in = *a.n_in;
    // the static tree's top levels, one copy per block
    const int n_top = kTop4 < a.st4.n_nodes ? kTop4 : a.st4.n_nodes;
    for (int k = threadIdx.x; k < n_top; k += blockDim.x) top[k] = a.st4.nodes[k];
    __syncthreads();
    unsigned s_nodes = 0, s_tris = 0, s_seg = 0, s_cap = 0, s_box4 = 0;
    // the first chunk of every wave is its own index (all waves start at
    // once, and a burst of atomics on one counter would serialise them); the
    // later ones come from the counter, after the grid's first chunks.
    const unsigned int n_waves = (gridDim.x * blockDim.x) >> 6;
    unsigned int chunk = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int rays_per_chunk = a.b >= 2 ? kBounceChunkLate : kBounceChunk;
    while (true) {
        unsigned long long base = (unsigned long long)chunk * (unsigned long long)rays_per_chunk;
        if (base >= n_in) break;
        for (int j = 0; j < rays_per_chunk; j += 64)
            bounce_chunk<STATS, REV>(a, n_in, base + (unsigned long long)j, lane, s_nodes, s_tris, s_seg, s_cap, s_box4,
                                     &stk, 64, top, n_top);
        unsigned int next = 0;
        if (lane == 0) next = atomicAdd(a.work, 1u);
        chunk = n_waves + (unsigned int)__shfl((int)next, 0);
    }
    flush_stats<STATS>(a.stats, lane, s_nodes, s_tris, s_seg, s_cap, s_box4);
}

// ------------------------------------------------- regroup between bounces ----
// Block b of the histogram and scatter kernels owns the rays [b n / B, (b+1) n / B)
// of the live buffer (B = gridDim.x, n read on the device).  Histogram rows are
// bin-major ([bin][block]), so one exclusive scan gives every (bin, block) its
// first output slot.
int regroup_blocks(long long n_total) {
    long long b = n_total / 4096;
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

size_t regroup_temp_u32(long long n_total) {
    const long long n = (long long)kRegroupBins * regroup_blocks(n_total);
    return (size_t)(2 * n + 64) + scan_temp_bytes(n) / 4 + 64;
}

__device__ __forceinline__ void block_range(const unsigned long long* n_dev, long long& beg, long long& end) {
    const long long n = (long long)*n_dev, nb = gridDim.x;
    beg = n * (long long)blockIdx.x / nb;
    end = n * ((long long)blockIdx.x + 1) / nb;
}

__global__ void __launch_bounds__(256) k_regroup_hist(const uint16_t* key, const unsigned long long* n_dev,
                                                      uint32_t* hist) {
    __shared__ uint32_t h[kRegroupBins];
    for (int k = threadIdx.x; k < kRegroupBins; k += blockDim.x) h[k] = 0u;
    __syncthreads();
    long long beg, end;
    block_range(n_dev, beg, end);
    for (long long i = beg + threadIdx.x; i < end; i += blockDim.x) atomicAdd(&h[key[i]], 1u);
    __syncthreads();
    for (int k = threadIdx.x; k < kRegroupBins; k += blockDim.x) hist[(long long)k * gridDim.x + blockIdx.x] = h[k];
}

__global__ void __launch_bounds__(256) k_regroup_scatter(RaySoA src, RaySoA dst, const uint16_t* key,
                                                         const unsigned long long* n_dev, const uint32_t* off) {
    __shared__ uint32_t cur[kRegroupBins];
    for (int k = threadIdx.x; k < kRegroupBins; k += blockDim.x) cur[k] = off[(long long)k * gridDim.x + blockIdx.x];
    __syncthreads();
    long long beg, end;
    block_range(n_dev, beg, end);
    for (long long i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const long long o = atomicAdd(&cur[key[i]], 1u);
        dst.ox[o] = src.ox[i]; dst.oy[o] = src.oy[i]; dst.oz[o] = src.oz[i];
        dst.dx[o] = src.dx[i]; dst.dy[o] = src.dy[i]; dst.dz[o] = src.dz[i];
        dst.L[o] = src.L[i];
        dst.id[o] = src.id[i];
        dst.prev[o] = src.prev[i];
    }
}

void regroup(const RaySoA& src, const RaySoA& dst, const uint16_t* key, const unsigned long long* n_dev, long long cap,
             uint32_t* temp, hipStream_t st) {
    const int nb = regroup_blocks(cap);
    const long long n = (long long)kRegroupBins * nb;
    uint32_t* hist = temp;
    uint32_t* off = hist + n;
    uint32_t* stemp = off + n + 64;
    hipLaunchKernelGGL(k_regroup_hist, dim3(nb), dim3(256), 0, st, key, n_dev, hist);
    exclusive_scan(hist, off, n, stemp, nullptr, st);
    hipLaunchKernelGGL(k_regroup_scatter, dim3(nb), dim3(256), 0, st, src, dst, key, n_dev, off);
}

void bounce(const BounceArgs& a, bool stats, int grid, hipStream_t st) {
    const bool rev = a.src.src_rx != nullptr;
    if (rev) {
        if (stats) hipLaunchKernelGGL((k_bounce<true, true>), dim3(grid), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_bounce<false, true>), dim3(grid), dim3(256), 0, st, a);
    } else {
        if (stats) hipLaunchKernelGGL((k_bounce<true, false>), dim3(grid), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_bounce<false, false>), dim3(grid), dim3(256), 0, st, a);
    }
}

// Several scenes in one launch (batched stepping): chunk_off[c] is the first
// global chunk of scene c (an exclusive scan of its live-ray chunks, built on
// the device by k_chunk_table); a wave takes the next global chunk, finds its
// scene by binary search and runs that scene's bounce on it.  A chunk holds
// `chunk` rays (32, 64, 128, 256, 512 or 1024): a wave traces them 64 at a
// time (32: with half its lanes), so larger chunks take fewer counter atomics
// and binary searches, smaller ones balance the tail better.
__global__ void __launch_bounds__(256) k_chunk_table(const BounceArgs* __restrict__ args, int n_scenes,
                                                     uint32_t* chunk_off, uint32_t* work, int chunk) {
    __shared__ uint32_t sh[256];
    uint32_t carry = 0;
    for (int base = 0; base < n_scenes; base += 256) {
        int c = base + (int)threadIdx.x;
        uint32_t v = c < n_scenes ? (uint32_t)((*args[c].n_in + (unsigned long long)chunk - 1ULL) /
                                               (unsigned long long)chunk)
                                  : 0u;
        sh[threadIdx.x] = v;
        __syncthreads();
        // inclusive Hillis-Steele scan of 256 values
        for (int o = 1; o < 256; o <<= 1) {
            uint32_t y = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0u;
            __syncthreads();
            sh[threadIdx.x] += y;
            __syncthreads();
        }
        if (c < n_scenes) chunk_off[c] = carry + sh[threadIdx.x] - v;
        carry += sh[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        chunk_off[n_scenes] = carry;
        *work = 0u;
    }
}

__global__ void __launch_bounds__(256) k_bounce_multi(const BounceArgs* __restrict__ args,
                                                      const uint32_t* __restrict__ chunk_off, uint32_t* work,
                                                      int n_scenes, int chunk) {
    __shared__ int stk_lds[kStackRows][kStackStride];
    LdsStack stk{&stk_lds[0][threadIdx.x]};
    const int lane = lane_id();
    const uint32_t total = chunk_off[n_scenes];
    unsigned s_nodes = 0, s_tris = 0, s_seg = 0, s_cap = 0, s_box4 = 0;
    // first chunk: the wave's own index; later ones from the counter
    const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
    uint32_t g = (uint32_t)__builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    for (bool first = true;; first = false) {
        if (!first) {
            uint32_t next = 0;
            if (lane == 0) next = atomicAdd(work, 1u);
            g = n_waves + (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)next, 0));
        }
        if (g >= total) break;
        int lo = 0, hi = n_scenes - 1;  // last scene with chunk_off[c] <= g
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (chunk_off[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        const int c = __builtin_amdgcn_readfirstlane(lo);
        const BounceArgs& a = args[c];
        const unsigned long long n_in = *a.n_in;
        // a chunk of `chunk` rays: 64 per pass (32: half the lanes)
        const unsigned long long base = (unsigned long long)(g - chunk_off[c]) * (unsigned long long)chunk;
        for (int j = 0; j < chunk; j += 64)
            bounce_chunk<false, false>(a, n_in, base + (unsigned long long)j, lane, s_nodes, s_tris, s_seg, s_cap,
                                       s_box4, &stk, chunk < 64 ? chunk : 64);
    }
}

void bounce_multi(const BounceArgs* args, int n_scenes, uint32_t* chunk_off, uint32_t* work, int grid, int chunk,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_chunk_table, dim3(1), dim3(256), 0, st, args, n_scenes, chunk_off, work, chunk);
    hipLaunchKernelGGL(k_bounce_multi, dim3(grid), dim3(256), 0, st, args, chunk_off, work, n_scenes, chunk);
}

// Hit log of launch direction i of transmitter tx (slot_of[i]: its launch
// slot); rows after the bounce at which the ray ended read -2.
__global__ void k_debug_rays(const int* hitlog, const uint8_t* depth, long long n_total, int K, int tx, int N,
                             const uint32_t* slot_of, const int* ids, int n, int* out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int i = ids[k];
    const long long ray = (i >= 0 && i < N) ? (long long)tx * N + slot_of[i] : -1;
    const int last = ray >= 0 ? (int)depth[ray] : -1;
    for (int b = 0; b <= K; b++)
        out[(long long)k * (K + 1) + b] = ray < 0 ? -3 : (b <= last ? hitlog[(long long)b * n_total + ray] : -2);
}

void debug_rays(const int* hitlog, const uint8_t* depth, long long n_total, int K, int tx, int N,
                const uint32_t* slot_of, const int* ray_ids, int n, int* out, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_debug_rays, dim3((n + 255) / 256), dim3(256), 0, st, hitlog, depth, n_total, K,
                                  tx, N, slot_of, ray_ids, n, out);
}

__global__ void k_invert_perm(const uint32_t* perm, uint32_t* inv, int n) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) inv[perm[t]] = (uint32_t)t;
}

void invert_perm(const uint32_t* perm, uint32_t* inv, int n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_invert_perm, dim3((n + 255) / 256), dim3(256), 0, st, perm, inv, n);
}

__global__ void k_debug_mark(uint32_t* sel, int tx, int N, const uint32_t* slot_of, const int* ids, int n,
                             uint32_t* bad) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int i = ids[k];
    if (i < 0 || i >= N) {
        atomicOr(bad, 1u);
        return;
    }
    const long long slot = (long long)tx * N + slot_of[i];
    atomicOr(&sel[slot >> 5], 1u << (slot & 31));
}

void debug_mark(uint32_t* sel, int tx, int N, const uint32_t* slot_of, const int* ray_ids, int n, uint32_t* bad,
                hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_debug_mark, dim3((n + 255) / 256), dim3(256), 0, st, sel, tx, N, slot_of, ray_ids,
                                  n, bad);
}

__global__ void k_debug_captures(const int* log, const unsigned long long* n_log, long long log_cap, int N,
                                 const uint32_t* perm, int* out, long long cap) {
    long long n = (long long)*n_log;
    if (n > log_cap) n = log_cap;
    if (n > cap) n = cap;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const long long slot = (unsigned)log[3 * k];
        const int tx = (int)(slot / N);
        out[5 * k] = tx;
        out[5 * k + 1] = (int)perm[slot - (long long)tx * N];
        out[5 * k + 2] = log[3 * k + 1] & 0xff;
        out[5 * k + 3] = log[3 * k + 1] >> 8;
        out[5 * k + 4] = log[3 * k + 2];
    }
}

void debug_captures(const int* log, const unsigned long long* n_log, long long log_cap, int N, const uint32_t* perm,
                    int* out, long long cap, hipStream_t st) {
    const long long g = (std::min(log_cap, cap) + 255) / 256;
    hipLaunchKernelGGL(k_debug_captures, dim3((unsigned)std::max(1LL, std::min(g, 4096LL))), dim3(256), 0, st, log,
                       n_log, log_cap, N, perm, out, cap);
}

}  // namespace emrt
