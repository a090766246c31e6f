// emrt_dev.h -- device-side data layouts and inline helpers of the gfx950
// dynamic SBR EM ray tracer (Wang & Manocha 2023, Sections II-A, III-B/C).
//
// Layouts (all device memory, coalesced SoA where threads stream):
//   BNode  64 B  internal node of a binary LBVH; both child boxes inline so a
//                node visit is four 16-byte loads; leaves are primitives.
//   TriP   48 B  triangle in leaf order: v0.xyz|tri id, v1.xyz|face, v2.xyz
//   KeyRec 32 B  path key: tx, rx, type|order<<8, ids[5] (faces or edge)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define EMRT_LEAF 0x80000000u
#define EMRT_SIDE 0x80000000u
#define EMRT_KMAX 5
#define EMRT_NF 4

namespace emrt {

constexpr double kPi = 3.14159265358979323846;
constexpr double kC0 = 299792458.0;

// --------------------------------------------------------------------------
// structures
// --------------------------------------------------------------------------
struct __attribute__((aligned(16))) BNode {
    float4 a;  // lmin.x lmin.y lmin.z lmax.x
    float4 b;  // lmax.y lmax.z rmin.x rmin.y
    float4 c;  // rmin.z rmax.x rmax.y rmax.z
    int4 m;    // left, right (EMRT_LEAF|slot for leaves), parent|side<<31, split axis
};

struct __attribute__((aligned(16))) TriP {
    float4 v0;  // w = tri id (int bits)
    float4 v1;  // w = face id (int bits)
    float4 v2;
};

struct KeyRec {
    int tx, rx, to;  // to = type | order << 8
    int ids[5];
};

// path types: line of sight, specular (ids = faces), edge diffraction
// (ids[0] = edge), reflection then diffraction (ids = face, edge) and
// diffraction then reflection (ids = edge, face)
enum { KT_LOS = 0, KT_SPEC = 1, KT_DIFF = 2, KT_RD = 3, KT_DR = 4 };

// device status flags (read back on sync)
enum : uint32_t {
    FLAG_TABLE_FULL = 1u << 0,
    FLAG_CAND_CAP = 1u << 1,
    FLAG_PATH_CAP = 1u << 2,
    FLAG_BAD_INPUT = 1u << 3,
    FLAG_NONFINITE = 1u << 4,
    FLAG_EDGE_CAP = 1u << 5,
};

struct Bvh {
    const BNode* nodes;
    int n_prims;  // 0: empty tree
};

// 4-wide node with quantised child boxes (the static tree, collapsed from
// its binary SAH tree): child k's box on axis a is
//   [fma(qlo, s_a, o_a), fma(qhi, s_a, o_a)],  s_a = 2^(e_a - 127) (0 when e_a = 0),
// with byte k of q.{x,y,z} / r.{x,y,z} holding child k's qlo / qhi on x, y,
// z.  The bytes are chosen at build time with the same fused multiply-add,
// so every decoded box contains its child's box.  64 B, one node per four
// children instead of two.
struct __attribute__((aligned(16))) QNode4 {
    float4 o;  // x, y, z: the node's low corner; w (bits): e_x | e_y << 8 | e_z << 16 | children << 24
    uint4 q;   // qlo bytes (x, y, z; w unused)
    uint4 r;   // qhi bytes (x, y, z; w unused)
    int4 c;    // children: node index, or EMRT_LEAF | primitive slot
};

struct Bvh4 {
    const QNode4* nodes;
    int n_prims;  // 0: empty tree
    int n_nodes;
};

// Depth of the 4-wide tree's top that the builder numbers breadth first
// (levels 0 .. kBvh4TopLevels, at most 85 nodes) and the bounce kernel keeps
// in LDS: every ray starts at the root, so these nodes are read by every
// query, and from LDS their loads do not wait on the cache hierarchy.
#ifndef EMRT_TOP4_LEVELS
#define EMRT_TOP4_LEVELS 3
#endif
constexpr int kBvh4TopLevels = EMRT_TOP4_LEVELS;
#ifndef EMRT_TOP4
#define EMRT_TOP4 85
#endif
constexpr int kTop4 = EMRT_TOP4;  // nodes staged (1 + 4 + 16 + 64 = 85)

// --------------------------------------------------------------------------
// float / double vectors
// --------------------------------------------------------------------------
struct dv3 { double x, y, z; };
__device__ __forceinline__ dv3 d3(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ dv3 operator+(dv3 a, dv3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ dv3 operator-(dv3 a, dv3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ dv3 operator*(dv3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ double dot(dv3 a, dv3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ dv3 cross(dv3 a, dv3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double len(dv3 a) { return sqrt(dot(a, a)); }
__device__ __forceinline__ dv3 unit(dv3 a) { return a * (1.0 / len(a)); }
__device__ __forceinline__ dv3 ldd3(const double* p) { return {p[0], p[1], p[2]}; }
__device__ __forceinline__ dv3 ldf3(const float* p) { return {(double)p[0], (double)p[1], (double)p[2]}; }

// --------------------------------------------------------------------------
// complex double
// --------------------------------------------------------------------------
struct cd { double re, im; };
__device__ __forceinline__ cd C(double r, double i = 0.0) { return {r, i}; }
__device__ __forceinline__ cd operator+(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd operator*(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd operator*(cd a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ cd cdiv(cd a, cd b) {
    // Smith's algorithm
    if (fabs(b.re) >= fabs(b.im)) {
        double r = b.im / b.re, den = b.re + b.im * r;
        return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
    }
    double r = b.re / b.im, den = b.im + b.re * r;
    return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}
__device__ __forceinline__ double cabs2(cd a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ double cabsd(cd a) { return hypot(a.re, a.im); }
__device__ __forceinline__ cd cexpi(double ph) { double s, c; sincos(ph, &s, &c); return {c, s}; }
// principal square root (Re >= 0)
__device__ __forceinline__ cd csqrtd(cd z) {
    double r = hypot(z.re, z.im);
    if (r == 0.0) return {0.0, 0.0};
    if (z.re >= 0.0) {
        double t = sqrt(0.5 * (r + z.re));
        return {t, z.im / (2.0 * t)};
    }
    double t = sqrt(0.5 * (r - z.re));
    return {fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

// --------------------------------------------------------------------------
// path keys and the open-addressing table
//   table slot (u64): 0 empty;
//     1<<62 | order<<59 | rx<<32 | ray       ray capture (order 1..7, rx < 2^27)
//     2<<62 | cache index                     key copied from the path cache
//     3<<62 | tx<<50 | edge<<26 | rx          diffraction candidate
// --------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}
__device__ __forceinline__ uint64_t key_hash(int tx, int rx, int to, const int* ids) {
    uint64_t h = mix64(((uint64_t)(uint32_t)tx << 32) ^ (uint64_t)(uint32_t)rx ^ 0x9E3779B97F4A7C15ULL);
    h = mix64(h ^ (uint64_t)(uint32_t)to);
    int type = to & 0xff, order = to >> 8;
    int n = type == KT_SPEC ? order : (type == KT_DIFF ? 1 : (type >= KT_RD ? 2 : 0));
    for (int j = 0; j < n; j++) h = mix64(h ^ ((uint64_t)(uint32_t)ids[j] + 0x632BE59BD9B4E019ULL * (uint64_t)(j + 1)));
    return h;
}
__device__ __forceinline__ uint64_t ref_ray(int order, int rx, uint32_t ray) {
    return (1ULL << 62) | ((uint64_t)order << 59) | ((uint64_t)rx << 32) | (uint64_t)ray;
}
__device__ __forceinline__ uint64_t ref_cache(uint32_t idx) { return (2ULL << 62) | (uint64_t)idx; }
// a key stored in the step's extra-key array (reflection-diffraction candidates)
__device__ __forceinline__ uint64_t ref_extra(uint32_t idx) { return (2ULL << 62) | (1ULL << 61) | (uint64_t)idx; }
__device__ __forceinline__ uint64_t ref_diff(int tx, int e, int rx) {
    return (3ULL << 62) | ((uint64_t)tx << 50) | ((uint64_t)e << 26) | (uint64_t)rx;
}

// Context needed to expand a table reference into its key.  A ray reference
// holds (order, target, ray id); the launch's source is ray / rays_per_tx.
// From the transmitters (src_rx null) the target is a receiver and the faces
// are in launch order; from receivers (src_rx[source] = receiver index) the
// target is a transmitter and the faces are taken in reverse, so the key is
// the same transmitter-to-receiver path either way.
struct KeySrc {
    const int* hitlog;     // [K+1][n_total] triangle id per bounce
    const int* tri_face;   // [T]
    const KeyRec* cache;   // previous cache
    long long n_total;     // rays in the launch
    int rays_per_tx;       // rays per source
    const int* src_rx;     // receiver-side launch: receiver of each source; null otherwise
    const KeyRec* extra;   // keys proposed by the reflection-diffraction candidates
};

// SIDE: 0 transmitter-side launch, 1 receiver-side, -1 read from s.src_rx
// (the bounce kernel, which knows its side, keeps the other branch out).
template <int SIDE = -1>
__device__ __forceinline__ void expand_ref(uint64_t ref, const KeySrc& s, KeyRec& k) {
    uint32_t tag = (uint32_t)(ref >> 62);
    if (tag == 1) {
        uint32_t ray = (uint32_t)ref;
        int order = (int)((ref >> 59) & 7);
        int source = (int)(ray / (uint32_t)s.rays_per_tx);
        int target = (int)((ref >> 32) & 0x7FFFFFF);
        k.to = KT_SPEC | (order << 8);
        if (SIDE == 1 || (SIDE < 0 && s.src_rx)) {
            k.tx = target;
            k.rx = s.src_rx[source];
            for (int j = 0; j < 5; j++)
                k.ids[j] = j < order ? s.tri_face[s.hitlog[(long long)(order - 1 - j) * s.n_total + ray]] : -1;
        } else {
            k.tx = source;
            k.rx = target;
            for (int j = 0; j < 5; j++)
                k.ids[j] = j < order ? s.tri_face[s.hitlog[(long long)j * s.n_total + ray]] : -1;
        }
    } else if (tag == 2) {
        k = (ref >> 61) & 1 ? s.extra[(uint32_t)(ref & 0x1FFFFFFFFFFFFFFFULL)]
                            : s.cache[(uint32_t)(ref & 0x1FFFFFFFFFFFFFFFULL)];
    } else {
        k.tx = (int)((ref >> 50) & 0xFFF);
        k.rx = (int)(ref & 0x3FFFFFF);
        k.to = KT_DIFF | (1 << 8);
        k.ids[0] = (int)((ref >> 26) & 0xFFFFFF);
        for (int j = 1; j < 5; j++) k.ids[j] = -1;
    }
}

__device__ __forceinline__ bool key_eq(const KeyRec& a, const KeyRec& b) {
    if (a.tx != b.tx || a.rx != b.rx || a.to != b.to) return false;
    for (int j = 0; j < 5; j++)
        if (a.ids[j] != b.ids[j]) return false;
    return true;
}

// lexicographic (tx, rx, type, order, ids) -- the within-link path order
__device__ __forceinline__ bool key_less(const KeyRec& a, const KeyRec& b) {
    if (a.tx != b.tx) return a.tx < b.tx;
    if (a.rx != b.rx) return a.rx < b.rx;
    int ta = a.to & 0xff, tb = b.to & 0xff;
    if (ta != tb) return ta < tb;
    int oa = a.to >> 8, ob = b.to >> 8;
    if (oa != ob) return oa < ob;
    for (int j = 0; j < 5; j++)
        if (a.ids[j] != b.ids[j]) return a.ids[j] < b.ids[j];
    return false;
}

// Set of (source, face, edge) triples lit by second segments (a ray that
// reflected off `face` passed the edge): 16 + 24 + 24 bits, bit 63 marks a
// used slot.  Returns false when the set is full.
__device__ __forceinline__ uint64_t pair_key(int source, int face, int edge) {
    return (1ULL << 63) | ((uint64_t)(uint32_t)source << 48) | ((uint64_t)(uint32_t)face << 24) | (uint64_t)(uint32_t)edge;
}
__device__ __forceinline__ bool pair_insert(unsigned long long* set, uint64_t mask, uint64_t key) {
    uint64_t slot = mix64(key) & mask;
    for (uint64_t probe = 0; probe <= mask; probe++) {
        unsigned long long cur = __hip_atomic_load(&set[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == key) return true;
        if (cur == 0ULL) {
            unsigned long long prev = atomicCAS(&set[slot], 0ULL, (unsigned long long)key);
            if (prev == 0ULL || prev == key) return true;
        }
        slot = (slot + 1) & mask;
    }
    return false;
}

// Insert `ref` whose expanded key is `mine` with hash h.  Returns 1 when
// inserted, 0 when an equal key is present, -1 when the table is full.
// Lock-free: a slot is claimed by one 64-bit CAS holding the whole
// reference, whose key data were written before this kernel started.
template <int SIDE = -1>
__device__ __forceinline__ int table_insert(unsigned long long* table, uint64_t mask, uint64_t ref, const KeyRec& mine,
                                            uint64_t h, const KeySrc& src) {
    uint64_t slot = h & mask;
    for (uint64_t probe = 0; probe <= mask; probe++) {
        unsigned long long cur = __hip_atomic_load(&table[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == 0ULL) {
            unsigned long long prev = atomicCAS(&table[slot], 0ULL, (unsigned long long)ref);
            if (prev == 0ULL) return 1;
            cur = prev;
        }
        if (cur == ref) return 0;
        KeyRec other;
        expand_ref<SIDE>(cur, src, other);
        if (key_eq(other, mine)) return 0;
        slot = (slot + 1) & mask;
    }
    return -1;
}

// Whether a key equal to `mine` (hash h) is in the table: a read-only probe
// (the table is not written while it runs).  Ray references always expand to
// specular keys, so other keys skip them without reading the hit log.
template <int SIDE = -1>
__device__ __forceinline__ bool table_find(const unsigned long long* table, uint64_t mask, const KeyRec& mine,
                                           uint64_t h, const KeySrc& src) {
    const bool spec = (mine.to & 0xff) == KT_SPEC;
    uint64_t slot = h & mask;
    for (uint64_t probe = 0; probe <= mask; probe++) {
        const unsigned long long cur = table[slot];
        if (cur == 0ULL) return false;
        if (spec || (cur >> 62) != 1ULL) {
            KeyRec other;
            expand_ref<SIDE>(cur, src, other);
            if (key_eq(other, mine)) return true;
        }
        slot = (slot + 1) & mask;
    }
    return false;
}

// --------------------------------------------------------------------------
// rays: precomputation for the slab test and the watertight triangle test
// (Woop, Benthin & Wald, "Watertight ray/triangle intersection", JCGT 2013)
// --------------------------------------------------------------------------
struct RayPre {
    float ox, oy, oz;
    float dx, dy, dz;
    float ix, iy, iz;  // 1/d (zero components replaced by +-1e-30)
    int kx, ky, kz;
    float Sx, Sy, Sz;
    int negmask;  // bit k set when d[k] < 0
    // -o/d per axis pushed down (nm) and up (np) by 8 ulps of its magnitude, for
    // the fused slab test: p/d - o/d evaluated as fma(p, 1/d, -o/d) stays
    // conservative (see slab_fma)
    float nmx, nmy, nmz, npx, npy, npz;
};

__device__ __forceinline__ float nz(float v) { return v != 0.0f ? v : 1e-30f; }

__device__ __forceinline__ RayPre ray_pre(float ox, float oy, float oz, float dx, float dy, float dz) {
    RayPre r;
    r.ox = ox; r.oy = oy; r.oz = oz;
    r.dx = dx; r.dy = dy; r.dz = dz;
    r.ix = 1.0f / nz(dx);
    r.iy = 1.0f / nz(dy);
    r.iz = 1.0f / nz(dz);
    r.negmask = (dx < 0.0f ? 1 : 0) | (dy < 0.0f ? 2 : 0) | (dz < 0.0f ? 4 : 0);
    float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    float dkz = kz == 0 ? dx : (kz == 1 ? dy : dz);
    if (dkz < 0.0f) { int t = kx; kx = ky; ky = t; }
    float dkx = kx == 0 ? dx : (kx == 1 ? dy : dz);
    float dky = ky == 0 ? dx : (ky == 1 ? dy : dz);
    r.kx = kx; r.ky = ky; r.kz = kz;
    r.Sx = dkx / dkz;
    r.Sy = dky / dkz;
    r.Sz = 1.0f / dkz;
    {
#pragma clang fp contract(off)
        const float qx = -(ox * r.ix), qy = -(oy * r.iy), qz = -(oz * r.iz);
        // 8 ulps (2^-21 |q|, an exact scaling) cover the rounding of q and of q -+ e
        const float ex = fabsf(qx) * 0x1p-21f, ey = fabsf(qy) * 0x1p-21f, ez = fabsf(qz) * 0x1p-21f;
        r.nmx = qx - ex; r.nmy = qy - ey; r.nmz = qz - ez;
        r.npx = qx + ex; r.npy = qy + ey; r.npz = qz + ez;
    }
    return r;
}

__device__ __forceinline__ float sel3(int k, float x, float y, float z) { return k == 0 ? x : (k == 1 ? y : z); }

// Conservative slab test (Ize, "Robust BVH ray traversal", JCGT 2013): far
// distance scaled by 1 + 2 gamma_3 so rounding never rejects a box that the
// exact ray touches.  Returns the entry distance through tn.
__device__ __forceinline__ bool slab(float lx, float ly, float lz, float hx, float hy, float hz, const RayPre& r,
                                     float tmin, float tmax, float& tn) {
    float t0x = (lx - r.ox) * r.ix, t1x = (hx - r.ox) * r.ix;
    float t0y = (ly - r.oy) * r.iy, t1y = (hy - r.oy) * r.iy;
    float t0z = (lz - r.oz) * r.iz, t1z = (hz - r.oz) * r.iz;
    float a = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), tmin));
    float b = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z)) * 1.0000003576278687f;
    tn = a;
    return a <= fminf(b, tmax);
}

// Conservative slab test with fused multiply-adds, for the closest-hit
// traversal.  The plane the ray meets first on an axis is the low one when
// the direction component is positive (the high one otherwise), so per axis
// one entry and one exit distance are computed, as fma(p, 1/d, -o/d -+ e):
// with e = 8 ulps of |o/d| the entry is at most t (1 + 3u) + ... below and the
// exit at least t (1 - 3u) (u = 2^-24, t the exact distance along the ray of
// the rounded inverse, as in the plain form), so scaling the exit bound
// (and the current closest distance) by 1 + 2^-20 never rejects a box the
// exact ray meets before that distance.  Returns the entry distance in tn.
__device__ __forceinline__ bool slab_fma(float lx, float ly, float lz, float hx, float hy, float hz, const RayPre& r,
                                         float tmax, float& tn) {
    const bool sx = r.negmask & 1, sy = r.negmask & 2, sz = r.negmask & 4;
    const float nx = fmaf(sx ? hx : lx, r.ix, r.nmx), fx = fmaf(sx ? lx : hx, r.ix, r.npx);
    const float ny = fmaf(sy ? hy : ly, r.iy, r.nmy), fy = fmaf(sy ? ly : hy, r.iy, r.npy);
    const float nz = fmaf(sz ? hz : lz, r.iz, r.nmz), fz = fmaf(sz ? lz : hz, r.iz, r.npz);
    const float a = fmaxf(fmaxf(nx, ny), fmaxf(nz, 0.0f));
    const float b = fminf(fminf(fx, fy), fminf(fz, tmax)) * 1.00000095367431640625f;  // 1 + 2^-20
    tn = a;
    return a <= b;
}

// Watertight ray/triangle test, two-sided; hit when t > 0.  Edge functions
// are evaluated without contraction so neighbouring triangles see exactly
// opposite values on a shared edge; zero edge functions are re-evaluated in
// double.
__device__ __forceinline__ bool tri_hit(const TriP& p, const RayPre& r, float& t_out) {
#pragma clang fp contract(off)
    float Ax0 = p.v0.x - r.ox, Ay0 = p.v0.y - r.oy, Az0 = p.v0.z - r.oz;
    float Bx0 = p.v1.x - r.ox, By0 = p.v1.y - r.oy, Bz0 = p.v1.z - r.oz;
    float Cx0 = p.v2.x - r.ox, Cy0 = p.v2.y - r.oy, Cz0 = p.v2.z - r.oz;
    float Akz = sel3(r.kz, Ax0, Ay0, Az0), Bkz = sel3(r.kz, Bx0, By0, Bz0), Ckz = sel3(r.kz, Cx0, Cy0, Cz0);
    float Ax = sel3(r.kx, Ax0, Ay0, Az0) - r.Sx * Akz;
    float Ay = sel3(r.ky, Ax0, Ay0, Az0) - r.Sy * Akz;
    float Bx = sel3(r.kx, Bx0, By0, Bz0) - r.Sx * Bkz;
    float By = sel3(r.ky, Bx0, By0, Bz0) - r.Sy * Bkz;
    float Cx = sel3(r.kx, Cx0, Cy0, Cz0) - r.Sx * Ckz;
    float Cy = sel3(r.ky, Cx0, Cy0, Cz0) - r.Sy * Ckz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        double u = (double)Cx * (double)By - (double)Cy * (double)Bx;
        double v = (double)Ax * (double)Cy - (double)Ay * (double)Cx;
        double w = (double)Bx * (double)Ay - (double)By * (double)Ax;
        U = (float)u; V = (float)v; W = (float)w;
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = U + V + W;
    if (det == 0.0f) return false;
    float Az = r.Sz * Akz, Bz = r.Sz * Bkz, Cz = r.Sz * Ckz;
    float T = U * Az + V * Bz + W * Cz;
    float t = T / det;
    if (!(t > 0.0f)) return false;
    t_out = t;
    return true;
}

// --------------------------------------------------------------------------
// BVH traversal
//
// Main loop: a short per-ray stack.  At an internal node both child boxes
// are tested; the nearer child is entered and the other pushed.  Each
// internal node is loaded once.
//
// The stack holds kStackDepth node ids; it only holds the pending far
// children along the current path, and the LBVHs of a city are about 25
// levels deep.  The bounce and shadow kernels keep it in one column of a
// block-wide LDS array (LdsStack below); kernels without that LDS keep it in
// a private array (RegStack), where a deeper stack costs registers.  On the
// city's bounces 10 and 12 entries ran alike and 16 or 20 cost about 6%; at
// 12 a restart is rare (0.0001% more node visits than with no overflow).  If
// a deeper tree overflows it, the traversal starts over with the walk over
// parent links below, which needs no stack; all queries are idempotent
// (closest hit with a fixed tie rule, any hit, leaf visits whose effects are
// set inserts), so work done before the restart does not change the result.
// --------------------------------------------------------------------------
#ifndef EMRT_STACK_DEPTH
#define EMRT_STACK_DEPTH 12
#endif
constexpr int kStackDepth = EMRT_STACK_DEPTH;
// The 4-wide tree pushes up to three children per level; its stack (the
// same LDS columns) holds 16 entries.
constexpr int kStackDepth4 = 16;
constexpr int kStackRows = kStackDepth4 > kStackDepth ? kStackDepth4 : kStackDepth;

__device__ __forceinline__ BNode ld_node(const BNode* n, int i) { return n[i]; }

__device__ __forceinline__ void child_box(const BNode& nd, int side, float& lx, float& ly, float& lz, float& hx,
                                          float& hy, float& hz, int& child) {
    if (side == 0) { lx = nd.a.x; ly = nd.a.y; lz = nd.a.z; hx = nd.a.w; hy = nd.b.x; hz = nd.b.y; child = nd.m.x; }
    else { lx = nd.b.z; ly = nd.b.w; lz = nd.c.x; hx = nd.c.y; hy = nd.c.z; hz = nd.c.w; child = nd.m.y; }
}

__device__ __forceinline__ int near_side(const BNode& nd, const RayPre& r) {
    int axis = nd.m.w & 3;
    return (r.negmask >> axis) & 1;
}

// The per-ray stack of node ids.  A private array indexed by each lane's own
// depth compiles to a chain of compares and selects over all its entries at
// every push and pop; kernels that can spare the LDS hand the traversal one
// column of a [kStackDepth][kStackStride] block array instead (one LDS access
// per push or pop; lanes of a wave sit in distinct banks at any depths).
struct RegStack {
    int s[kStackDepth];
    __device__ __forceinline__ int get(int i) const { return s[i]; }
    __device__ __forceinline__ void set(int i, int v) { s[i] = v; }
};
constexpr int kStackStride = 256;  // threads per block of the kernels that use LdsStack
struct LdsStack {
    int* p;  // &column[0][threadIdx.x]
    __device__ __forceinline__ int get(int i) const { return p[i * kStackStride]; }
    __device__ __forceinline__ void set(int i, int v) { p[i * kStackStride] = v; }
};

// Stackless walk over parent links.  State per ray: the current internal
// node and what is left to do there: 0 test the first child, 1 test the
// second child, 2 climb to the parent, 3 just climbed back from child `came`
// (decides between 1 and 2).
template <bool ORDERED, class Test, class Stop>
__device__ __forceinline__ void traverse_stackless(const BNode* nodes, const RayPre& r, Test test, Stop stop) {
    int cur = 0, state = 0, came = 0;
    while (true) {
        BNode nd = ld_node(nodes, cur);
        int first = ORDERED ? near_side(nd, r) : 0;
        if (state == 3) state = (came == first) ? 1 : 2;
        bool descended = false;
        float tn;
        if (state == 0) {
            int child;
            float lx, ly, lz, hx, hy, hz;
            child_box(nd, first, lx, ly, lz, hx, hy, hz, child);
            if (test(lx, ly, lz, hx, hy, hz, child, tn)) { cur = child; descended = true; }
            else state = 1;
            if (stop()) return;
        }
        if (!descended && state == 1) {
            int child;
            float lx, ly, lz, hx, hy, hz;
            child_box(nd, 1 - first, lx, ly, lz, hx, hy, hz, child);
            if (test(lx, ly, lz, hx, hy, hz, child, tn)) { cur = child; state = 0; descended = true; }
            else state = 2;
            if (stop()) return;
        }
        if (descended) continue;
        if (cur == 0) return;
        uint32_t pz = (uint32_t)nd.m.z;
        came = (int)(pz >> 31);
        cur = (int)(pz & 0x7FFFFFFFu);
        state = ORDERED ? 3 : (came ? 2 : 1);
    }
}

// Generic driver.  test(box, child, tn) returns true to descend into `child`
// (an internal node; tn = the box's entry distance); it handles leaves itself
// and returns false for them.  Returns early when stop() is true.
template <bool ORDERED, class Stk, class Test, class Stop>
__device__ __forceinline__ void traverse_with(const BNode* nodes, const RayPre& r, Test test, Stop stop, Stk& stk) {
    int sp = 0, cur = 0;
    bool overflow = false;
    while (true) {
        BNode nd = ld_node(nodes, cur);
        // both boxes in stored order (no per-lane selection of box fields),
        // then the near one first
        float l0, l1;
        bool d0 = test(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, nd.m.x, l0);
        if (stop()) return;
        bool d1 = test(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, nd.m.y, l1);
        if (stop()) return;
        const int first = ORDERED ? near_side(nd, r) : 0;
        const int ca = first ? nd.m.y : nd.m.x, cb = first ? nd.m.x : nd.m.y;
        const bool da = first ? d1 : d0, db = first ? d0 : d1;
        if (da) {
            if (db) {
                if (sp == kStackDepth) { overflow = true; break; }
                stk.set(sp, cb);
                sp++;
            }
            cur = ca;
            continue;
        }
        if (db) {
            cur = cb;
            continue;
        }
        if (sp == 0) return;
        cur = stk.get(--sp);
    }
    if (overflow) traverse_stackless<ORDERED>(nodes, r, test, stop);
}

// stk null: a private register stack
template <bool ORDERED, class Stk, class Test, class Stop>
__device__ __forceinline__ void traverse(const BNode* nodes, const RayPre& r, Test test, Stop stop, Stk* stk) {
    if constexpr (std::is_same<Stk, RegStack>::value) {
        RegStack own;
        traverse_with<ORDERED>(nodes, r, test, stop, own);
    } else {
        traverse_with<ORDERED>(nodes, r, test, stop, *stk);
    }
}

struct NoStop { __device__ bool operator()() const { return false; } };

// One leaf triangle of the closest-hit query (ties to the lowest triangle id).
template <bool STATS>
__device__ __forceinline__ void leaf_closest(const TriP* prims, int child, const RayPre& r, int skip_face,
                                             float& best_t, int& best_tri, int& best_face, unsigned& n_tris) {
    TriP p = prims[(int)((uint32_t)child & ~EMRT_LEAF)];
    if (STATS) n_tris++;
    int face = __float_as_int(p.v1.w);
    float t;
    // the test runs whatever the face (it has no side effects), so the whole
    // primitive is fetched in one round trip instead of the face id first
    const bool h = tri_hit(p, r, t);
    if (h && face != skip_face) {
        int id = __float_as_int(p.v0.w);
        if (t < best_t || (t == best_t && id < best_tri)) { best_t = t; best_tri = id; best_face = face; }
    }
}

// Closest hit with the query-independent generic traversal (the fallback of
// closest_hit when its short stack overflows).
template <bool STATS, class Stk = RegStack>
__device__ __forceinline__ void closest_hit_generic(const Bvh& bvh, const TriP* prims, const RayPre& r, int skip_face,
                                                    float& best_t, int& best_tri, int& best_face, unsigned& n_nodes,
                                                    unsigned& n_tris, Stk* stk = nullptr) {
    if (bvh.n_prims <= 0) return;
    traverse<true>(bvh.nodes, r,
        [&](float lx, float ly, float lz, float hx, float hy, float hz, int child, float& tn) -> bool {
            if (!slab(lx, ly, lz, hx, hy, hz, r, 0.0f, best_t, tn)) return false;
            if (!((uint32_t)child & EMRT_LEAF)) { if (STATS) n_nodes++; return true; }
            TriP p = prims[(int)((uint32_t)child & ~EMRT_LEAF)];
            if (STATS) n_tris++;
            int face = __float_as_int(p.v1.w);
            float t;
            if (face != skip_face && tri_hit(p, r, t)) {
                int id = __float_as_int(p.v0.w);
                if (t < best_t || (t == best_t && id < best_tri)) { best_t = t; best_tri = id; best_face = face; }
            }
            return false;
        },
        NoStop(), stk);
}

// Closest hit among triangles not on face `skip_face`.  best_t / best_tri /
// best_face carry the current best (ties broken by the lowest triangle id),
// so the result does not depend on the tree or the visiting order.
//
// Per node: both child boxes by the fused slab test (no branch), then the
// leaf children that the ray meets (at most two triangles), then the
// internal children: the one with the nearer entry is entered and the other
// pushed.  Each node is loaded once.  If the short stack overflows, the query
// starts over with the generic traversal, which needs no stack.
template <bool STATS, class Stk = RegStack>
__device__ __forceinline__ void closest_hit(const Bvh& bvh, const TriP* prims, const RayPre& r, int skip_face,
                                            float& best_t, int& best_tri, int& best_face, unsigned& n_nodes,
                                            unsigned& n_tris, Stk* stk = nullptr) {
    if (bvh.n_prims <= 0) return;
    if (STATS) n_nodes++;
    RegStack own;
    int sp = 0, cur = 0;
    bool overflow = false;
    while (true) {
        const BNode nd = ld_node(bvh.nodes, cur);
        float t0, t1;
        const bool d0 = slab_fma(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, r, best_t, t0);
        const bool d1 = slab_fma(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, r, best_t, t1);
        const int c0 = nd.m.x, c1 = nd.m.y;
        const bool leaf0 = (uint32_t)c0 & EMRT_LEAF, leaf1 = (uint32_t)c1 & EMRT_LEAF;
        if ((d0 && leaf0) || (d1 && leaf1)) {
            if (d0 && leaf0) leaf_closest<STATS>(prims, c0, r, skip_face, best_t, best_tri, best_face, n_tris);
            if (d1 && leaf1) leaf_closest<STATS>(prims, c1, r, skip_face, best_t, best_tri, best_face, n_tris);
        }
        const bool i0 = d0 && !leaf0, i1 = d1 && !leaf1;
        if (STATS) n_nodes += (i0 ? 1u : 0u) + (i1 ? 1u : 0u);
        const bool second = i1 && (!i0 || t1 < t0);  // enter child 1 first
        const int ca = second ? c1 : c0, cb = second ? c0 : c1;
        if (i0 && i1) {
            if (sp == kStackDepth) { overflow = true; break; }
            if constexpr (std::is_same<Stk, RegStack>::value) own.set(sp, cb);
            else stk->set(sp, cb);
            sp++;
        }
        if (i0 || i1) {
            cur = ca;
            continue;
        }
        if (sp == 0) break;
        --sp;
        if constexpr (std::is_same<Stk, RegStack>::value) cur = own.get(sp);
        else cur = stk->get(sp);
    }
    if (overflow) closest_hit_generic<STATS>(bvh, prims, r, skip_face, best_t, best_tri, best_face, n_nodes, n_tris, stk);
}


// Any hit on the open segment t in (0, tmax) among triangles not on faces
// xa / xb / xc (shadow rays of path validation).
template <class Stk = RegStack>
__device__ __forceinline__ bool any_hit(const Bvh& bvh, const TriP* prims, const RayPre& r, float tmax, int xa, int xb,
                                        int xc = -1, Stk* stk = nullptr) {
    if (bvh.n_prims <= 0) return false;
    bool found = false;
    traverse<true>(bvh.nodes, r,
        [&](float lx, float ly, float lz, float hx, float hy, float hz, int child, float& tn) -> bool {
            if (!slab(lx, ly, lz, hx, hy, hz, r, 0.0f, tmax, tn)) return false;
            if (!((uint32_t)child & EMRT_LEAF)) return true;
            TriP p = prims[(int)((uint32_t)child & ~EMRT_LEAF)];
            int face = __float_as_int(p.v1.w);
            float t;
            if (face != xa && face != xb && face != xc && tri_hit(p, r, t) && t < tmax) found = true;
            return false;
        },
        [&]() { return found; }, stk);
    return found;
}

// Child k of a 4-wide node: decoded box (exact fma of the stored bytes, as at
// build time) through the fused slab test.
// The byte words of a node's entry and exit planes for this ray: on an axis
// where the ray runs backwards the entry plane is the high one.  Chosen once
// per node for all four children (the per-child choice of slab_fma, hoisted).
struct Planes4 {
    uint32_t ex, ey, ez;  // entry-plane bytes (child k in byte k)
    uint32_t fx, fy, fz;  // exit-plane bytes
};
__device__ __forceinline__ Planes4 planes4(const QNode4& nd, const RayPre& r) {
    const bool sx = r.negmask & 1, sy = r.negmask & 2, sz = r.negmask & 4;
    return Planes4{sx ? nd.r.x : nd.q.x, sy ? nd.r.y : nd.q.y, sz ? nd.r.z : nd.q.z,
                   sx ? nd.q.x : nd.r.x, sy ? nd.q.y : nd.r.y, sz ? nd.q.z : nd.r.z};
}

// Child K's box against the ray: the same decode (fma of the byte with the
// axis scale, onto the node's corner) and fused slab test as slab_fma.
template <int K>
__device__ __forceinline__ bool child4(const QNode4& nd, const Planes4& pl, float sx, float sy, float sz,
                                       const RayPre& r, float tmax, float& tn) {
    const float nx = fmaf(fmaf((float)((pl.ex >> (8 * K)) & 255u), sx, nd.o.x), r.ix, r.nmx);
    const float ny = fmaf(fmaf((float)((pl.ey >> (8 * K)) & 255u), sy, nd.o.y), r.iy, r.nmy);
    const float nz = fmaf(fmaf((float)((pl.ez >> (8 * K)) & 255u), sz, nd.o.z), r.iz, r.nmz);
    const float fx = fmaf(fmaf((float)((pl.fx >> (8 * K)) & 255u), sx, nd.o.x), r.ix, r.npx);
    const float fy = fmaf(fmaf((float)((pl.fy >> (8 * K)) & 255u), sy, nd.o.y), r.iy, r.npy);
    const float fz = fmaf(fmaf((float)((pl.fz >> (8 * K)) & 255u), sz, nd.o.z), r.iz, r.npz);
    const float a = fmaxf(fmaxf(nx, ny), fmaxf(nz, 0.0f));
    const float b = fminf(fminf(fx, fy), fminf(fz, tmax)) * 1.00000095367431640625f;  // 1 + 2^-20
    tn = a;
    return a <= b;
}

__device__ __forceinline__ float scale4(uint32_t bits, int shift) {
    return __int_as_float((int)(((bits >> shift) & 255u) << 23));
}

// compare-exchange of (entry distance, child) pairs, nearer first
__device__ __forceinline__ void cx4(float& ta, int& ca, float& tb, int& cb) {
    const bool sw = tb < ta;
    const float t = sw ? tb : ta;
    const int c = sw ? cb : ca;
    tb = sw ? ta : tb;
    cb = sw ? ca : cb;
    ta = t;
    ca = c;
}

// Closest hit over a 4-wide tree (same query, result and tie rule as
// closest_hit): the boxes of a node's children are tested, leaf children
// (triangles) tested at once, and the internal children the ray meets are
// sorted by entry distance: the nearest is entered and the others pushed so
// that they pop nearest first.  A stack overflow restarts the query on the
// binary tree `bin` with the generic traversal (same result).
// STATS: n_boxes counts the child boxes tested (a node's children), n_nodes
// the binary nodes of a fallback traversal.
// top: copies of the nodes [0, n_top) (in LDS), read in place of bvh.nodes.
template <bool STATS, class Stk>
__device__ __forceinline__ void closest_hit4(const Bvh4& bvh, const Bvh& bin, const TriP* prims, const RayPre& r,
                                             int skip_face, float& best_t, int& best_tri, int& best_face,
                                             unsigned& n_boxes, unsigned& n_nodes, unsigned& n_tris, Stk* stk,
                                             const QNode4* top = nullptr, int n_top = 0) {
    if (bvh.n_prims <= 0) return;
    int sp = 0, cur = 0;
    bool overflow = false;
    while (true) {
        QNode4 nd;
        if (cur < n_top) nd = top[cur];
        else nd = bvh.nodes[cur];
        const uint32_t meta = __float_as_uint(nd.o.w);
        const int cnt = (int)(meta >> 24);
        if (STATS) n_boxes += (unsigned)cnt;
        const float sx = scale4(meta, 0), sy = scale4(meta, 8), sz = scale4(meta, 16);
        const Planes4 pl = planes4(nd, r);
        float t0, t1, t2, t3;
        const bool h0 = child4<0>(nd, pl, sx, sy, sz, r, best_t, t0) && cnt > 0;
        const bool h1 = child4<1>(nd, pl, sx, sy, sz, r, best_t, t1) && cnt > 1;
        const bool h2 = child4<2>(nd, pl, sx, sy, sz, r, best_t, t2) && cnt > 2;
        const bool h3 = child4<3>(nd, pl, sx, sy, sz, r, best_t, t3) && cnt > 3;
        int c0 = nd.c.x, c1 = nd.c.y, c2 = nd.c.z, c3 = nd.c.w;
        // the leaf children the ray meets, tested one per pass of a loop over
        // this lane's own set: the wave runs the triangle test as many times
        // as its busiest lane needs, not once per child slot any lane needs
        unsigned lm = (h0 && c0 < 0 ? 1u : 0u) | (h1 && c1 < 0 ? 2u : 0u) | (h2 && c2 < 0 ? 4u : 0u) |
                      (h3 && c3 < 0 ? 8u : 0u);
#pragma unroll 1
        for (; lm; lm &= lm - 1u) {
            const int k = __builtin_ctz(lm);
            const int lo = (k & 1) ? c1 : c0, hi = (k & 1) ? c3 : c2;
            leaf_closest<STATS>(prims, (k & 2) ? hi : lo, r, skip_face, best_t, best_tri, best_face, n_tris);
        }
        // internal children met by the ray, by entry distance (others at +inf)
        t0 = (h0 && c0 >= 0) ? t0 : INFINITY;
        t1 = (h1 && c1 >= 0) ? t1 : INFINITY;
        t2 = (h2 && c2 >= 0) ? t2 : INFINITY;
        t3 = (h3 && c3 >= 0) ? t3 : INFINITY;
        const int n_in = (t0 < INFINITY) + (t1 < INFINITY) + (t2 < INFINITY) + (t3 < INFINITY);
        if (n_in == 0) {
            if (sp == 0) break;
            cur = stk->get(--sp);
            continue;
        }
        cx4(t0, c0, t1, c1);
        cx4(t2, c2, t3, c3);
        cx4(t0, c0, t2, c2);
        cx4(t1, c1, t3, c3);
        cx4(t1, c1, t2, c2);
        if (sp + n_in - 1 > kStackDepth4) { overflow = true; break; }
        if (n_in > 3) stk->set(sp++, c3);
        if (n_in > 2) stk->set(sp++, c2);
        if (n_in > 1) stk->set(sp++, c1);
        cur = c0;
    }
    if (overflow) closest_hit_generic<STATS>(bin, prims, r, skip_face, best_t, best_tri, best_face, n_nodes, n_tris, stk);
}

// Any hit on the open segment t in (0, tmax) over a 4-wide tree among
// triangles not on faces xa / xb / xc (shadow rays).  Overflow restarts on
// the binary tree.
template <class Stk>
__device__ __forceinline__ bool any_hit4(const Bvh4& bvh, const Bvh& bin, const TriP* prims, const RayPre& r,
                                         float tmax, int xa, int xb, int xc, Stk* stk) {
    if (bvh.n_prims <= 0) return false;
    int sp = 0, cur = 0;
    while (true) {
        const QNode4 nd = bvh.nodes[cur];
        const uint32_t meta = __float_as_uint(nd.o.w);
        const int cnt = (int)(meta >> 24);
        const float sx = scale4(meta, 0), sy = scale4(meta, 8), sz = scale4(meta, 16);
        const Planes4 pl = planes4(nd, r);
        float t0, t1, t2, t3;
        const bool h0 = child4<0>(nd, pl, sx, sy, sz, r, tmax, t0) && cnt > 0;
        const bool h1 = child4<1>(nd, pl, sx, sy, sz, r, tmax, t1) && cnt > 1;
        const bool h2 = child4<2>(nd, pl, sx, sy, sz, r, tmax, t2) && cnt > 2;
        const bool h3 = child4<3>(nd, pl, sx, sy, sz, r, tmax, t3) && cnt > 3;
        const int cs[4] = {nd.c.x, nd.c.y, nd.c.z, nd.c.w};
        const bool hs[4] = {h0, h1, h2, h3};
        bool found = false;
        // leaf children met, one per pass over this lane's own set (as in closest_hit4)
        unsigned lm = (h0 && cs[0] < 0 ? 1u : 0u) | (h1 && cs[1] < 0 ? 2u : 0u) | (h2 && cs[2] < 0 ? 4u : 0u) |
                      (h3 && cs[3] < 0 ? 8u : 0u);
#pragma unroll 1
        for (; lm; lm &= lm - 1u) {
            const int k = __builtin_ctz(lm);
            const int lo = (k & 1) ? cs[1] : cs[0], hi = (k & 1) ? cs[3] : cs[2];
            TriP p = prims[(int)((uint32_t)((k & 2) ? hi : lo) & ~EMRT_LEAF)];
            const int face = __float_as_int(p.v1.w);
            float t;
            const bool h = tri_hit(p, r, t);  // whatever the face: one fetch of the primitive
            if (h && face != xa && face != xb && face != xc && t < tmax) found = true;
        }
        if (found) return true;
        int next = -1;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (hs[k] && cs[k] >= 0) {
                if (next < 0) next = cs[k];
                else {
                    if (sp == kStackDepth4) return any_hit(bin, prims, r, tmax, xa, xb, xc, stk);
                    stk->set(sp++, cs[k]);
                }
            }
        }
        if (next >= 0) {
            cur = next;
            continue;
        }
        if (sp == 0) return false;
        cur = stk->get(--sp);
    }
}

// Visit every leaf whose box, inflated by `grow`, meets the ray on [0, tmax].
template <class Leaf, class Stk = RegStack>
__device__ __forceinline__ void all_hits(const Bvh& bvh, const RayPre& r, float tmax, float grow, Leaf leaf,
                                         Stk* stk = nullptr) {
    if (bvh.n_prims <= 0) return;
    traverse<false>(bvh.nodes, r,
        [&](float lx, float ly, float lz, float hx, float hy, float hz, int child, float& tn) -> bool {
            if (!slab(lx - grow, ly - grow, lz - grow, hx + grow, hy + grow, hz + grow, r, 0.0f, tmax, tn)) return false;
            if (!((uint32_t)child & EMRT_LEAF)) return true;
            leaf((int)((uint32_t)child & ~EMRT_LEAF));
            return false;
        },
        NoStop(), stk);
}

// Visit every leaf whose box overlaps the query box [ql, qh].
template <class Leaf>
__device__ __forceinline__ void box_query(const Bvh& bvh, float qlx, float qly, float qlz, float qhx, float qhy,
                                          float qhz, Leaf leaf) {
    if (bvh.n_prims <= 0) return;
    RayPre dummy{};
    traverse<false>(bvh.nodes, dummy,
        [&](float lx, float ly, float lz, float hx, float hy, float hz, int child, float& tn) -> bool {
            tn = 0.0f;
            bool ov = lx <= qhx && hx >= qlx && ly <= qhy && hy >= qly && lz <= qhz && hz >= qlz;
            if (!ov) return false;
            if (!((uint32_t)child & EMRT_LEAF)) return true;
            leaf((int)((uint32_t)child & ~EMRT_LEAF));
            return false;
        },
        NoStop(), (RegStack*)nullptr);
}

// wave helpers (wave64)
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
__device__ __forceinline__ uint64_t ballot64(bool p) { return (uint64_t)__ballot(p); }
__device__ __forceinline__ int prefix_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
// one atomic per wave: returns this lane's slot in a compacted output
__device__ __forceinline__ long long wave_append(unsigned long long* counter, bool keep) {
    uint64_t m = ballot64(keep);
    int cnt = __popcll(m);
    unsigned long long base = 0;
    int leader = __ffsll((long long)m) - 1;
    if (cnt > 0 && lane_id() == leader) base = atomicAdd(counter, (unsigned long long)cnt);
    base = __shfl(base, leader < 0 ? 0 : leader);
    return keep ? (long long)(base + (unsigned long long)prefix_below(m)) : -1;
}

// One atomic per wave for a variable number of items per lane: every lane of
// the wave calls this at the same point (uniform control flow); returns the
// lane's first slot.  Inclusive scan over the wave with shuffles.
__device__ __forceinline__ unsigned long long wave_reserve(unsigned long long* counter, uint32_t n) {
    const int lane = lane_id();
    uint32_t x = n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    uint32_t total = __shfl(x, 63);
    unsigned long long base = 0;
    if (lane == 63 && total > 0) base = atomicAdd(counter, (unsigned long long)total);
    base = __shfl(base, 63);
    return base + (unsigned long long)(x - n);
}

}  // namespace emrt
