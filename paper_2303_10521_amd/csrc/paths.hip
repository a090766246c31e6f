// paths.hip -- path cache, exact path validation, field evaluation and the
// per-receiver channel sums.
//
// Section II-A: propagation paths are cached to exploit temporal coherence;
// Section III-B: valid paths stay in the cache ("visibility hash table") and
// are deleted once invalid.  Every frame the cached keys (and, on discovery
// frames, the keys found by the rays) are rebuilt exactly: image method over
// the face planes for reflections, Keller's law for first-order edge
// diffraction, float32 shadow rays through the LBVHs for every leg.
// Fields are evaluated in double (Fresnel reflection of the tracked
// polarisation, UTD for diffraction), with the delay and the Doppler shift of
// Section III-C (Eq (3) generalised to moving interaction points) and the
// power-weighted mean Doppler shift / RMS Doppler spread of Section V-D.
#include "emrt_dev.h"
#include "emrt_launch.h"
#include "fields.h"

namespace emrt {

#define GRID_STRIDE(i, n) for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

static int grid_for(long long n, int block = 256, int cap = 8192) {
    long long g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ------------------------------------------------- temporal coherence ----
// The static tree is built once per scene.  A key whose end points did not
// move since the last step and whose faces (and edge) are static has the
// same legs as then, so its tests against the static tree give the same
// answers: a key valid at the last step is clear of the static scene, and a
// line of sight the static scene blocked is still blocked.  Only the dynamic
// tree is tested for such keys; everything else is tested in full.
__global__ void k_endpoints_moved(const double* pos, double* prev, int n, uint8_t* moved, const uint32_t* hist) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const bool same = *hist && x == prev[3 * i] && y == prev[3 * i + 1] && z == prev[3 * i + 2];
    moved[i] = same ? 0 : 1;
    prev[3 * i] = x;
    prev[3 * i + 1] = y;
    prev[3 * i + 2] = z;
}

void endpoints_moved(const double* pos, double* prev, int n, uint8_t* moved, const uint32_t* hist, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_endpoints_moved, dim3((n + 255) / 256), dim3(256), 0, st, pos, prev, n, moved, hist);
}

__device__ __forceinline__ bool key_static(const SceneDev& S, const KeyRec& key) {
    const int type = key.to & 0xff, order = key.to >> 8;
    if (type == KT_SPEC) {
        bool st = true;
#pragma unroll
        for (int j = 0; j < EMRT_KMAX; j++)
            if (j < order && S.face_dyn[key.ids[j]] >= 0) st = false;
        return st;
    }
    if (type == KT_DIFF) return S.face_dyn[S.edge_i[6 * (long long)key.ids[0] + 2]] < 0;
    if (type == KT_RD || type == KT_DR) {
        const int f = type == KT_RD ? key.ids[0] : key.ids[1], e = type == KT_RD ? key.ids[1] : key.ids[0];
        return S.face_dyn[f] < 0 && S.face_dyn[S.edge_i[6 * (long long)e + 2]] < 0;
    }
    return true;
}

// ------------------------------------------------------------- tables ----
__global__ void k_cache_insert(unsigned long long* table, unsigned long long mask, const KeyRec* cache,
                               const unsigned long long* n_cache, long long cap, KeySrc src, uint32_t* flags) {
    long long n = (long long)*n_cache;
    if (n > cap) n = cap;
    GRID_STRIDE(c, n) {
        KeyRec k = cache[c];
        uint64_t h = key_hash(k.tx, k.rx, k.to, k.ids);
        if (table_insert(table, mask, ref_cache((uint32_t)c), k, h, src) < 0) atomicOr(flags, FLAG_TABLE_FULL);
    }
}

void cache_insert(unsigned long long* table, unsigned long long mask, const KeyRec* cache,
                  const unsigned long long* n_cache, long long cap, KeySrc src, uint32_t* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_cache_insert, dim3(grid_for(cap)), dim3(256), 0, st, table, mask, cache, n_cache, cap, src,
                       flags);
}

// Table compaction without a shared counter, in slot order (cache
// references excepted, see emitted_ref).  Each wave owns
// kCompactSpan consecutive slots: a first pass counts its occupied slots, an
// exclusive scan of the per-wave counts gives every wave its first candidate
// index, and a second pass re-reads the slots and places each occupied one by
// a ballot prefix (the table is read twice; no per-slot flags or offsets).
constexpr int kCompactIters = 64;
constexpr long long kCompactSpan = 64LL * kCompactIters;

// Cache references stay in the table (they make the rays' and the diffraction
// candidates' copies of cached keys duplicates) but are not emitted: the
// cache itself is appended in its own (link, key) order, which keeps
// neighbouring keys together for validation.
__device__ __forceinline__ bool emitted_ref(unsigned long long r) {
    return r != 0ULL && !((r >> 62) == 2ULL && !((r >> 61) & 1ULL));
}

__global__ void __launch_bounds__(256) k_slot_count(const unsigned long long* table, unsigned long long n_slots,
                                                    uint32_t* wave_cnt, long long n_waves) {
    const long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = (int)(threadIdx.x & 63);
    if (w >= n_waves) return;
    const long long base = w * kCompactSpan;
    uint32_t c = 0;
#pragma unroll 8
    for (int it = 0; it < kCompactIters; it++) {
        long long i = base + (long long)it * 64 + lane;
        c += (i < (long long)n_slots && emitted_ref(table[i])) ? 1u : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane == 0) wave_cnt[w] = c;
}

__global__ void __launch_bounds__(256) k_table_emit(const unsigned long long* table, unsigned long long n_slots,
                                                    const uint32_t* wave_off, long long n_waves, KeySrc src,
                                                    KeyRec* cand, long long cap, uint32_t* flags) {
    const long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = (int)(threadIdx.x & 63);
    if (w >= n_waves) return;
    const long long base = w * kCompactSpan;
    unsigned long long pos0 = wave_off[w];
    bool over = false;
    for (int it = 0; it < kCompactIters; it++) {
        long long i = base + (long long)it * 64 + lane;
        unsigned long long ref = i < (long long)n_slots ? table[i] : 0ULL;
        const bool emit = emitted_ref(ref);
        uint64_t m = ballot64(emit);
        if (emit) {
            long long pos = (long long)(pos0 + (unsigned long long)prefix_below(m));
            if (pos < cap) {
                KeyRec k;
                expand_ref(ref, src, k);
                cand[pos] = k;
            } else {
                over = true;
            }
        }
        pos0 += (unsigned long long)__popcll(m);
    }
    if (over) atomicOr(flags, FLAG_CAND_CAP);
}

long long compact_temp_elems(unsigned long long n_slots) {
    return ((long long)n_slots + kCompactSpan - 1) / kCompactSpan + 1;
}

void table_compact(const unsigned long long* table, unsigned long long n_slots, KeySrc src, KeyRec* cand,
                   unsigned long long* n_cand, long long cap, uint32_t* flags, const CompactTemp& t, hipStream_t st) {
    const long long n_waves = ((long long)n_slots + kCompactSpan - 1) / kCompactSpan;
    const int g = (int)((n_waves + 3) / 4);
    hipLaunchKernelGGL(k_slot_count, dim3(g), dim3(256), 0, st, table, n_slots, t.flags, n_waves);
    // n_cand: low word = scan total (its high word is cleared with the step's counters)
    exclusive_scan(t.flags, t.off, n_waves, t.scan_tmp, (uint32_t*)n_cand, st);
    hipLaunchKernelGGL(k_table_emit, dim3(g), dim3(256), 0, st, table, n_slots, t.off, n_waves, src, cand, cap,
                       flags);
}

// ------------------------------------------------------------ geometry ----

__device__ __forceinline__ dv3 mirror(dv3 p, const double* pl) {
#pragma clang fp contract(off)
    dv3 n = d3(pl[0], pl[1], pl[2]);
    return p - n * (2.0 * (dot(n, p) - pl[3]));
}

// point-in-triangle after dropping the dominant normal axis (edges inside)
__device__ __forceinline__ bool in_tri(dv3 p, dv3 a, dv3 b, dv3 c) {
#pragma clang fp contract(off)
    dv3 n = cross(b - a, c - a);
    double ax = fabs(n.x), ay = fabs(n.y), az = fabs(n.z);
    double P0, P1, A0, A1, B0, B1, C0, C1;
    if (az >= ax && az >= ay) { P0 = p.x; P1 = p.y; A0 = a.x; A1 = a.y; B0 = b.x; B1 = b.y; C0 = c.x; C1 = c.y; }
    else if (ay >= ax) { P0 = p.z; P1 = p.x; A0 = a.z; A1 = a.x; B0 = b.z; B1 = b.x; C0 = c.z; C1 = c.x; }
    else { P0 = p.y; P1 = p.z; A0 = a.y; A1 = a.z; B0 = b.y; B1 = b.z; C0 = c.y; C1 = c.z; }
    double w0 = (B0 - P0) * (C1 - P1) - (B1 - P1) * (C0 - P0);
    double w1 = (C0 - P0) * (A1 - P1) - (C1 - P1) * (A0 - P0);
    double w2 = (A0 - P0) * (B1 - P1) - (A1 - P1) * (B0 - P0);
    return (w0 >= 0 && w1 >= 0 && w2 >= 0) || (w0 <= 0 && w1 <= 0 && w2 <= 0);
}

// Lowest triangle id of face f containing p, or -1.
//
// Faces of at most kFaceLinearMax triangles are scanned in id order
// (face_tris is sorted by id within a face, so the first hit is the lowest;
// face_tv holds the world vertices of face_tris[q] at 9 q), after a reject
// against the face's bounding box: a point farther than 1e-6 m (+ 1e-9 of
// the coordinate) outside it cannot be accepted, since the points tested lie
// on the face plane up to double rounding and the triangle test accepts
// points of the triangle only up to that rounding.
//
// Larger faces (a tiled ground) are searched through the triangle LBVH of
// their kind (static or dynamic): every triangle of the face whose box
// overlaps p +- 1 mm is tested and the lowest accepted id kept, which is the
// same triangle the scan in id order would find.  The search uses the
// caller's LDS traversal stack.
constexpr int kFaceLinearMax = 32;

__device__ __forceinline__ int face_contains(const PathArgs& a, int f, dv3 p, LdsStack* stk) {
    const SceneDev& s = a.s;
    const int q0 = s.face_off[f], q1 = s.face_off[f + 1];
    if (q1 - q0 <= kFaceLinearMax) {
        const float* bx = s.face_box + 6 * (long long)f;
        const double pc[3] = {p.x, p.y, p.z};
#pragma unroll
        for (int c = 0; c < 3; c++) {
            double m = 1e-6 + 1e-9 * fabs(pc[c]);
            if (pc[c] < (double)bx[c] - m || pc[c] > (double)bx[3 + c] + m) return -1;
        }
        for (int q = q0; q < q1; q++) {
            const float* v = s.face_tv + 9 * (long long)q;
            if (in_tri(p, ldf3(v), ldf3(v + 3), ldf3(v + 6))) return s.face_tris[q];
        }
        return -1;
    }
    const bool dyn = s.face_dyn[f] >= 0;
    const Bvh t = dyn ? a.dy : a.st;
    const TriP* prims = dyn ? a.dy_prims : a.st_prims;
    if (t.n_prims <= 0) return -1;
    const float qlx = (float)(p.x - 1e-3), qly = (float)(p.y - 1e-3), qlz = (float)(p.z - 1e-3);
    const float qhx = (float)(p.x + 1e-3), qhy = (float)(p.y + 1e-3), qhz = (float)(p.z + 1e-3);
    int found = -1;
    RayPre dummy{};
    traverse<false>(t.nodes, dummy,
        [&](float lx, float ly, float lz, float hx, float hy, float hz, int child, float& tn) -> bool {
            tn = 0.0f;
            if (!(lx <= qhx && hx >= qlx && ly <= qhy && hy >= qly && lz <= qhz && hz >= qlz)) return false;
            if (!((uint32_t)child & EMRT_LEAF)) return true;
            TriP tp = prims[(int)((uint32_t)child & ~EMRT_LEAF)];
            if (__float_as_int(tp.v1.w) != f) return false;
            int id = __float_as_int(tp.v0.w);
            if (found >= 0 && id > found) return false;
            dv3 v0 = d3(tp.v0.x, tp.v0.y, tp.v0.z), v1 = d3(tp.v1.x, tp.v1.y, tp.v1.z), v2 = d3(tp.v2.x, tp.v2.y, tp.v2.z);
            if (in_tri(p, v0, v1, v2)) found = id;
            return false;
        },
        NoStop(), stk);
    return found;
}


// Keller point (equal angles with the edge) strictly inside the edge, both
// ends in the exterior wedge, receiver leg within diff_max_leg.  The source's
// share (its edge coordinates and wedge angle) is computed once per edge and
// reused for every receiver; the tests are the same pure expressions either
// way, so the outcome does not depend on the split or on their order.
struct KellerSrc {
    double zs, rs;
    bool ok;  // the source lies in the exterior wedge
};

__device__ __forceinline__ KellerSrc keller_src(const Wedge& w, dv3 s) {
#pragma clang fp contract(off)
    KellerSrc k;
    k.zs = dot(s - w.P0, w.e);
    k.rs = len(s - w.P0 - w.e * k.zs);
    double php = wedge_angle(w, s);
    k.ok = php > 0 && php < w.n * kPi;
    return k;
}

__device__ __forceinline__ bool keller_rx(const Wedge& w, const KellerSrc& k, dv3 r, double max_leg, dv3& Q) {
#pragma clang fp contract(off)
    if (!k.ok) return false;
    double zr = dot(r - w.P0, w.e);
    double rr = len(r - w.P0 - w.e * zr);
    if (!(k.rs + rr > 0)) return false;
    double zq = k.zs + (zr - k.zs) * k.rs / (k.rs + rr);
    if (!(zq > 0.0 && zq < w.len)) return false;
    Q = w.P0 + w.e * zq;
    if (!(len(Q - r) <= max_leg)) return false;
    double ph = wedge_angle(w, r);
    return ph > 0 && ph < w.n * kPi;
}

__device__ __forceinline__ bool keller(const Wedge& w, dv3 s, dv3 r, double max_leg, dv3& Q) {
    return keller_rx(w, keller_src(w, s), r, max_leg, Q);
}

// -------------------------------------------------------- diffraction ----
// Diffraction candidates: for every lit (tx, edge) pair, the receivers in the
// edge's box grown by diff_max_leg + 1 m, each tested exactly (Keller point
// strictly inside the edge, both ends in the exterior wedge, receiver leg
// within diff_max_leg) and inserted into the path table.
//
// The receivers are binned per frame on a kGridN x kGridN grid over their
// x-y bounding box (counting sort by cell), so the receivers of one row of
// cells are contiguous; one wave takes one lit pair and its lanes test the
// receivers of the overlapped rows in parallel, as one range over all the
// rows (a row holds a dozen receivers, far fewer than a wave's lanes).  Cell
// indices are monotone in the float32 coordinates, so the rows cover every
// receiver in the box.
__device__ __forceinline__ int grid_cell(float v, float v0, float inv_h) {
    float f = floorf((v - v0) * inv_h);
    if (!(f >= 0.0f)) return 0;  // also NaN
    return f > (float)(kGridN - 1) ? kGridN - 1 : (int)f;
}

__global__ void __launch_bounds__(256) k_rx_grid(const double* rx, int n, RxGrid* g) {
    __shared__ float sh[4][256];
    float lx = INFINITY, ly = INFINITY, hx = -INFINITY, hy = -INFINITY;
    for (int i = threadIdx.x; i < n; i += 256) {
        float x = (float)rx[3 * (long long)i], y = (float)rx[3 * (long long)i + 1];
        lx = fminf(lx, x); ly = fminf(ly, y); hx = fmaxf(hx, x); hy = fmaxf(hy, y);
    }
    sh[0][threadIdx.x] = lx; sh[1][threadIdx.x] = ly; sh[2][threadIdx.x] = hx; sh[3][threadIdx.x] = hy;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] = fminf(sh[0][threadIdx.x], sh[0][threadIdx.x + w]);
            sh[1][threadIdx.x] = fminf(sh[1][threadIdx.x], sh[1][threadIdx.x + w]);
            sh[2][threadIdx.x] = fmaxf(sh[2][threadIdx.x], sh[2][threadIdx.x + w]);
            sh[3][threadIdx.x] = fmaxf(sh[3][threadIdx.x], sh[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float ext = fmaxf(fmaxf(sh[2][0] - sh[0][0], sh[3][0] - sh[1][0]), 1.0f);
        if (!(ext < INFINITY)) ext = 1.0f;  // no receivers, or non-finite input (flagged elsewhere)
        g->x0 = sh[0][0] < INFINITY ? sh[0][0] : 0.0f;
        g->y0 = sh[1][0] < INFINITY ? sh[1][0] : 0.0f;
        g->inv_h = (float)kGridN / ext;
    }
}

__global__ void __launch_bounds__(256) k_rx_count(const double* rx, int n, const RxGrid* g, uint32_t* cnt) {
    const RxGrid gr = *g;
    GRID_STRIDE(i, (long long)n) {
        int cx = grid_cell((float)rx[3 * i], gr.x0, gr.inv_h), cy = grid_cell((float)rx[3 * i + 1], gr.y0, gr.inv_h);
        atomicAdd(&cnt[cy * kGridN + cx], 1u);
    }
}

__global__ void __launch_bounds__(256) k_rx_scatter(const double* rx, int n, const RxGrid* g, const uint32_t* start,
                                                    uint32_t* cursor, float4* sorted) {
    const RxGrid gr = *g;
    GRID_STRIDE(i, (long long)n) {
        float x = (float)rx[3 * i], y = (float)rx[3 * i + 1], z = (float)rx[3 * i + 2];
        int c = grid_cell(y, gr.y0, gr.inv_h) * kGridN + grid_cell(x, gr.x0, gr.inv_h);
        uint32_t pos = start[c] + atomicAdd(&cursor[c], 1u);
        sorted[pos] = make_float4(x, y, z, __int_as_float((int)i));
    }
}

void rx_grid_build(const double* rx_pos, int n_rx, const RxBins& b, hipStream_t st) {
    const long long nc = (long long)kGridN * kGridN;
    hipLaunchKernelGGL(k_rx_grid, dim3(1), dim3(256), 0, st, rx_pos, n_rx, b.grid);
    fill_u32(b.cnt, 0u, nc, st);
    fill_u32(b.cursor, 0u, nc, st);
    int g = grid_for(n_rx);
    hipLaunchKernelGGL(k_rx_count, dim3(g), dim3(256), 0, st, rx_pos, n_rx, b.grid, b.cnt);
    exclusive_scan(b.cnt, b.start, nc, b.scan_tmp, b.start + nc, st);
    hipLaunchKernelGGL(k_rx_scatter, dim3(g), dim3(256), 0, st, rx_pos, n_rx, b.grid, b.start, b.cursor, b.sorted);
}

// Transmitter-side diffraction candidates are unique by construction (one
// wave per lit (tx, edge), each receiver in exactly one grid cell), so they
// do not enter the path table: a lookup drops the ones the cache already
// holds, and the rest are appended to their own list in the order they are
// made.  That keeps the keys of one edge and nearby receivers together for
// the construction and shadow kernels (table slots are in hash order).  A
// wave stages its keys in LDS and reserves room for kStage of them at a time.
constexpr int kStage = 256;

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void stage_flush(unsigned long long* st, uint32_t& ns, const FreshKeys& fk, int lane,
                                            uint32_t* flags) {
    if (ns == 0u) return;
    wave_sync_lds();
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(fk.count, (unsigned long long)ns);
    base = __shfl(base, 0);
    bool over = false;
    for (uint32_t i = (uint32_t)lane; i < ns; i += 64u) {
        if (base + i < (unsigned long long)fk.cap) fk.ref[base + i] = st[i];
        else over = true;
    }
    if (over) atomicOr(flags, FLAG_CAND_CAP);
    ns = 0u;
    wave_sync_lds();
}

__global__ void __launch_bounds__(256) k_diff_cand(PathArgs a, const uint32_t* illum, int e_words, RxBins bins,
                                                   const unsigned long long* table, unsigned long long mask,
                                                   KeySrc src, FreshKeys fk) {
    __shared__ unsigned long long stage[4][kStage];
    const long long n = (long long)a.f.n_tx * a.s.E;
    const int lane = lane_id();
    unsigned long long* st = stage[threadIdx.x >> 6];
    uint32_t ns = 0;  // keys staged by this wave (wave-uniform)
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long n_waves = ((long long)gridDim.x * blockDim.x) >> 6;
    const RxGrid gr = *bins.grid;
    for (long long k = wave; k < n; k += n_waves) {
        int tx = (int)(k / a.s.E), e = (int)(k - (long long)tx * a.s.E);
        if (!(illum[(long long)tx * e_words + (e >> 5)] & (1u << (e & 31)))) continue;
        Wedge w = wedge_of(a.s, e);
        const KellerSrc ks = keller_src(w, ldd3(a.f.tx_pos + 3 * tx));
        if (!ks.ok) continue;  // no receiver can pass
        dv3 P1 = w.P0 + w.e * w.len;
        float g = (float)a.diff_max_leg + 1.0f;
        float qlx = (float)fmin(w.P0.x, P1.x) - g, qly = (float)fmin(w.P0.y, P1.y) - g, qlz = (float)fmin(w.P0.z, P1.z) - g;
        float qhx = (float)fmax(w.P0.x, P1.x) + g, qhy = (float)fmax(w.P0.y, P1.y) + g, qhz = (float)fmax(w.P0.z, P1.z) + g;
        int cx0 = grid_cell(qlx, gr.x0, gr.inv_h), cx1 = grid_cell(qhx, gr.x0, gr.inv_h);
        int cy0 = grid_cell(qly, gr.y0, gr.inv_h), cy1 = grid_cell(qhy, gr.y0, gr.inv_h);
        // up to 64 rows at a time: lane r holds row cy0 + r's receiver range;
        // the lanes then walk the rows' receivers as one flat range
        for (int rb = cy0; rb <= cy1; rb += 64) {
            const int cy = rb + lane;
            uint32_t j0 = 0, cnt = 0;
            if (cy <= cy1) {
                j0 = bins.start[cy * kGridN + cx0];
                cnt = bins.start[cy * kGridN + cx1 + 1] - j0;
            }
            uint32_t incl = cnt;  // inclusive prefix of the row counts
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                uint32_t y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            const uint32_t total = __shfl(incl, 63);
            for (uint32_t base = 0; base < total; base += 64u) {
                const uint32_t idx = base + (uint32_t)lane;
                int r = 0;  // the row holding flat index idx: rows whose prefix ends at or before it
#pragma unroll
                for (int sp = 32; sp >= 1; sp >>= 1) {
                    uint32_t v = __shfl(incl, r + sp - 1);
                    if (v <= idx) r += sp;
                }
                const uint32_t row_j0 = __shfl(j0, r), row_before = __shfl(incl - cnt, r);
                bool keep = false;
                int rx = 0;
                if (idx < total) {
                    float4 p = bins.sorted[row_j0 + (idx - row_before)];
                    rx = __float_as_int(p.w);
                    dv3 Q;
                    keep = p.x >= qlx && p.x <= qhx && p.y >= qly && p.y <= qhy && p.z >= qlz && p.z <= qhz &&
                           keller_rx(w, ks, ldd3(a.f.rx_pos + 3 * rx), a.diff_max_leg, Q);
                    if (keep) {
                        KeyRec key;
                        key.tx = tx; key.rx = rx; key.to = KT_DIFF | (1 << 8);
                        key.ids[0] = e; key.ids[1] = key.ids[2] = key.ids[3] = key.ids[4] = -1;
                        keep = !table_find(table, mask, key, key_hash(key.tx, key.rx, key.to, key.ids), src);
                    }
                }
                const uint64_t m = ballot64(keep);
                if (ns + (uint32_t)__popcll(m) > (uint32_t)kStage) stage_flush(st, ns, fk, lane, a.flags);
                if (keep) st[ns + (uint32_t)prefix_below(m)] = ref_diff(tx, e, rx);
                ns += (uint32_t)__popcll(m);
            }
        }
    }
    stage_flush(st, ns, fk, lane, a.flags);
}

// The fresh diffraction keys, expanded behind the table's candidates.
__global__ void __launch_bounds__(256) k_fresh_emit(FreshKeys fk, const unsigned long long* n_cand, KeyRec* cand,
                                                    long long cap, KeySrc src, uint32_t* flags) {
    long long nf = (long long)*fk.count;
    if (nf > fk.cap) nf = fk.cap;
    const long long base = (long long)*n_cand;
    GRID_STRIDE(i, nf) {
        const long long pos = base + i;
        if (pos < cap) {
            KeyRec k;
            expand_ref(fk.ref[i], src, k);
            cand[pos] = k;
        } else if (pos == cap || i == 0) {
            atomicOr(flags, FLAG_CAND_CAP);
        }
    }
}

__global__ void k_fresh_count(unsigned long long* n_cand, FreshKeys fk) {
    long long nf = (long long)*fk.count;
    if (nf > fk.cap) nf = fk.cap;
    *n_cand += (unsigned long long)nf;
}

// The previous cache behind the table's candidates, in its own order.
__global__ void __launch_bounds__(256) k_cache_emit(const KeyRec* cache, const unsigned long long* n_cache,
                                                    long long cap_cache, const unsigned long long* n_cand,
                                                    KeyRec* cand, long long cap, uint32_t* flags) {
    long long nc = (long long)*n_cache;
    if (nc > cap_cache) nc = cap_cache;
    const long long base = (long long)*n_cand;
    GRID_STRIDE(i, nc) {
        const long long pos = base + i;
        if (pos < cap) cand[pos] = cache[i];
        else if (pos == cap || i == 0) atomicOr(flags, FLAG_CAND_CAP);
    }
}

__global__ void k_cache_count(unsigned long long* n_cand, const unsigned long long* n_cache, long long cap_cache) {
    long long nc = (long long)*n_cache;
    if (nc > cap_cache) nc = cap_cache;
    *n_cand += (unsigned long long)nc;
}

void cache_append(const KeyRec* cache, const unsigned long long* n_cache, long long cap_cache,
                  unsigned long long* n_cand, KeyRec* cand, long long cap, uint32_t* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_cache_emit, dim3(grid_for(cap_cache)), dim3(256), 0, st, cache, n_cache, cap_cache, n_cand,
                       cand, cap, flags);
    hipLaunchKernelGGL(k_cache_count, dim3(1), dim3(1), 0, st, n_cand, n_cache, cap_cache);
}

void fresh_append(const FreshKeys& fk, unsigned long long* n_cand, KeyRec* cand, long long cap, KeySrc src,
                  uint32_t* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_fresh_emit, dim3(grid_for(fk.cap)), dim3(256), 0, st, fk, n_cand, cand, cap, src, flags);
    hipLaunchKernelGGL(k_fresh_count, dim3(1), dim3(1), 0, st, n_cand, fk);
}

void diff_candidates(const PathArgs& a, const uint32_t* illum, int e_words, const RxBins& bins,
                     const unsigned long long* table, unsigned long long mask, KeySrc src, const FreshKeys& fk,
                     hipStream_t st) {
    long long n = (long long)a.f.n_tx * a.s.E;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_diff_cand, dim3(grid_for(n, 4, 16384)), dim3(256), 0, st, a, illum, e_words, bins, table,
                       mask, src, fk);
}

// Edges lit from receivers (a receiver-side launch): one wave per lit
// (source, edge) pair, lanes over the transmitters; a transmitter whose Keller
// point on the edge passes the construction test becomes the candidate
// (tx, edge, receiver).
__global__ void __launch_bounds__(256) k_diff_cand_rx(PathArgs a, const uint32_t* illum, int e_words,
                                                      const int* src_rx, int n_src, unsigned long long* table,
                                                      unsigned long long mask, KeySrc src) {
    const long long n = (long long)n_src * a.s.E;
    const int lane = lane_id();
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long n_waves = ((long long)gridDim.x * blockDim.x) >> 6;
    for (long long k = wave; k < n; k += n_waves) {
        int q = (int)(k / a.s.E), e = (int)(k - (long long)q * a.s.E);
        if (!(illum[(long long)q * e_words + (e >> 5)] & (1u << (e & 31)))) continue;
        const int rx = src_rx[q];
        const Wedge w = wedge_of(a.s, e);
        const dv3 r = ldd3(a.f.rx_pos + 3 * rx);
        for (int tx = lane; tx < a.f.n_tx; tx += 64) {
            dv3 Q;
            if (!keller(w, ldd3(a.f.tx_pos + 3 * tx), r, a.diff_max_leg, Q)) continue;
            KeyRec key;
            key.tx = tx; key.rx = rx; key.to = KT_DIFF | (1 << 8);
            key.ids[0] = e; key.ids[1] = key.ids[2] = key.ids[3] = key.ids[4] = -1;
            uint64_t h = key_hash(key.tx, key.rx, key.to, key.ids);
            if (table_insert(table, mask, ref_diff(tx, e, rx), key, h, src) < 0) atomicOr(a.flags, FLAG_TABLE_FULL);
        }
    }
}

void diff_candidates_rx(const PathArgs& a, const uint32_t* illum, int e_words, const int* src_rx, int n_src,
                        unsigned long long* table, unsigned long long mask, KeySrc src, hipStream_t st) {
    long long n = (long long)n_src * a.s.E;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_diff_cand_rx, dim3(grid_for(n, 4, 16384)), dim3(256), 0, st, a, illum, e_words, src_rx,
                       n_src, table, mask, src);
}

// ---- one reflection and one diffraction --------------------------------
// The used slots of the pair set, listed (one atomic per wave).
__global__ void __launch_bounds__(256) k_pair_list(const unsigned long long* set, long long n,
                                                   unsigned long long* list, unsigned long long* count) {
    const long long lanes = (long long)gridDim.x * blockDim.x;
    const long long n_up = (n + 63) / 64 * 64;  // every lane of a wave takes the same trips
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_up; i += lanes) {
        const unsigned long long v = i < n ? set[i] : 0ULL;
        const long long pos = wave_append(count, v != 0ULL);
        if (v != 0ULL) list[pos] = v;
    }
}

// A proposed key goes into the extra-key array, then into the path table by
// reference (duplicates of cached keys leave their extra slot unused).
__device__ __forceinline__ void extra_insert(const ExtraKeys& xk, const KeyRec& key, unsigned long long* table,
                                             unsigned long long mask, const KeySrc& src, uint32_t* flags) {
    const unsigned long long i = atomicAdd(xk.count, 1ULL);
    if (i >= (unsigned long long)xk.cap) {
        atomicOr(flags, FLAG_CAND_CAP);
        return;
    }
    xk.key[i] = key;
    __threadfence();
    const uint64_t h = key_hash(key.tx, key.rx, key.to, key.ids);
    if (table_insert(table, mask, ref_extra((uint32_t)i), key, h, src) < 0) atomicOr(flags, FLAG_TABLE_FULL);
}

// One wave per listed (source, face, edge).  Transmitter-side launch (src_rx
// null): the transmitter's image in the face plane diffracts at the edge
// toward every receiver of the grid cells near the edge (reflection then
// diffraction).  Receiver-side launch: the receiver's image in the face plane
// receives the diffraction of every transmitter (diffraction then
// reflection).  The Keller test is the construction's own, so no valid path
// is lost.
__global__ void __launch_bounds__(256) k_pair_cand(PathArgs a, const unsigned long long* list,
                                                   const unsigned long long* n_list, RxBins bins, const int* src_rx,
                                                   ExtraKeys xk, unsigned long long* table, unsigned long long mask,
                                                   KeySrc src) {
    const long long n = (long long)*n_list;
    const int lane = lane_id();
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long n_waves = ((long long)gridDim.x * blockDim.x) >> 6;
    for (long long k = wave; k < n; k += n_waves) {
        const uint64_t v = list[k];
        const int source = (int)((v >> 48) & 0x7FFFULL), f = (int)((v >> 24) & 0xFFFFFFULL), e = (int)(v & 0xFFFFFFULL);
        if (f >= a.s.F || e >= a.s.E) continue;
        const Wedge w = wedge_of(a.s, e);
        if (f == w.f0 || f == w.fn) continue;
        const double* pl = a.s.plane + 4 * (long long)f;
        if (!src_rx) {
            if (source >= a.f.n_tx) continue;
            const RxGrid gr = *bins.grid;
            const dv3 img = mirror(ldd3(a.f.tx_pos + 3 * source), pl);
            dv3 P1 = w.P0 + w.e * w.len;
            float g = (float)a.diff_max_leg + 1.0f;
            float qlx = (float)fmin(w.P0.x, P1.x) - g, qly = (float)fmin(w.P0.y, P1.y) - g, qlz = (float)fmin(w.P0.z, P1.z) - g;
            float qhx = (float)fmax(w.P0.x, P1.x) + g, qhy = (float)fmax(w.P0.y, P1.y) + g, qhz = (float)fmax(w.P0.z, P1.z) + g;
            int cx0 = grid_cell(qlx, gr.x0, gr.inv_h), cx1 = grid_cell(qhx, gr.x0, gr.inv_h);
            int cy0 = grid_cell(qly, gr.y0, gr.inv_h), cy1 = grid_cell(qhy, gr.y0, gr.inv_h);
            for (int cy = cy0; cy <= cy1; cy++) {
                uint32_t j0 = bins.start[cy * kGridN + cx0], j1 = bins.start[cy * kGridN + cx1 + 1];
                for (uint32_t j = j0 + (uint32_t)lane; j < j1; j += 64u) {
                    float4 p = bins.sorted[j];
                    if (!(p.x >= qlx && p.x <= qhx && p.y >= qly && p.y <= qhy && p.z >= qlz && p.z <= qhz)) continue;
                    int rx = __float_as_int(p.w);
                    dv3 Q;
                    if (!keller(w, img, ldd3(a.f.rx_pos + 3 * rx), a.diff_max_leg, Q)) continue;
                    KeyRec key;
                    key.tx = source; key.rx = rx; key.to = KT_RD | (2 << 8);
                    key.ids[0] = f; key.ids[1] = e; key.ids[2] = key.ids[3] = key.ids[4] = -1;
                    extra_insert(xk, key, table, mask, src, a.flags);
                }
            }
        } else {
            const int rx = src_rx[source];
            const dv3 img = mirror(ldd3(a.f.rx_pos + 3 * rx), pl);
            for (int tx = lane; tx < a.f.n_tx; tx += 64) {
                dv3 Q;
                if (!keller(w, ldd3(a.f.tx_pos + 3 * tx), img, a.diff_max_leg, Q)) continue;
                KeyRec key;
                key.tx = tx; key.rx = rx; key.to = KT_DR | (2 << 8);
                key.ids[0] = e; key.ids[1] = f; key.ids[2] = key.ids[3] = key.ids[4] = -1;
                extra_insert(xk, key, table, mask, src, a.flags);
            }
        }
    }
}

void pair_candidates(const PathArgs& a, const unsigned long long* set, long long n_slots, unsigned long long* list,
                     unsigned long long* n_list, const RxBins& bins, const int* src_rx, const ExtraKeys& xk,
                     unsigned long long* table, unsigned long long mask, KeySrc src, hipStream_t st) {
    if (n_slots <= 0) return;
    hipLaunchKernelGGL(k_pair_list, dim3(grid_for(n_slots, 256, 4096)), dim3(256), 0, st, set, n_slots, list, n_list);
    hipLaunchKernelGGL(k_pair_cand, dim3(4096), dim3(256), 0, st, a, list, n_list, bins, src_rx, xk, table, mask,
                       src);
}

// Receiver positions of a receiver-side launch, gathered as its sources.
__global__ void k_gather_rx(const double* rx_pos, const int* sel, int n, double* out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int r = sel[i];
    out[3 * i] = rx_pos[3 * r];
    out[3 * i + 1] = rx_pos[3 * r + 1];
    out[3 * i + 2] = rx_pos[3 * r + 2];
}

void gather_rx(const double* rx_pos, const int* sel, int n, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_rx, dim3((n + 255) / 256), dim3(256), 0, st, rx_pos, sel, n, out);
}

// Geometry of one path key.  Points: P[0] = Tx, P[1..order] reflection
// points (or P[1] = Keller point), R = Rx; leg i runs from P[i] to P[i+1]
// (R for the last leg).  Loops run to the compile-time bound so every array
// index is a constant and the arrays stay in registers.
struct Built {
    dv3 P[EMRT_KMAX + 2];
    dv3 R;
    int order, type, np;  // np = number of points including Tx and Rx
    int tri[EMRT_KMAX];
    Wedge w;
};

__device__ __forceinline__ bool key_in_range(const PathArgs& a, const KeyRec& key) {
    int type = key.to & 0xff, order = key.to >> 8;
    bool good = key.tx >= 0 && key.tx < a.f.n_tx && key.rx >= 0 && key.rx < a.f.n_rx;
    if (type == KT_SPEC) {
        good = good && order >= 1 && order <= EMRT_KMAX;
#pragma unroll
        for (int j = 0; j < EMRT_KMAX; j++)
            if (j < order && !(key.ids[j] >= 0 && key.ids[j] < a.s.F)) good = false;
    } else if (type == KT_DIFF) {
        good = good && order == 1 && key.ids[0] >= 0 && key.ids[0] < a.s.E;
    } else if (type == KT_RD || type == KT_DR) {
        const int f = type == KT_RD ? key.ids[0] : key.ids[1], e = type == KT_RD ? key.ids[1] : key.ids[0];
        good = good && a.combined && order == 2 && f >= 0 && f < a.s.F && e >= 0 && e < a.s.E;
    } else if (type != KT_LOS) {
        good = false;
    }
    return good;
}

// Exact construction (everything except occlusion):
//   line of sight: the segment Tx -> Rx;
//   specular (image method): images s_k = mirror(s_{k-1}, plane f_k), then
//   back from Rx, x_k = segment(x_{k+1} -> s_k) meets plane f_k at a
//   parameter in (0, 1) and lies in a triangle of f_k (lowest id reported);
//   diffraction: Keller point strictly inside the edge, both ends in the
//   exterior wedge, receiver leg within diff_max_leg;
//   reflection then diffraction / diffraction then reflection: the same with
//   the image of Tx / of Rx in the face plane, plus the reflection point's
//   parameter in (0, 1) and its face (not a face of the wedge).
__device__ __forceinline__ bool construct(const PathArgs& a, const KeyRec& key, Built& g, LdsStack* stk) {
#pragma clang fp contract(off)
    const SceneDev& S = a.s;
    g.type = key.to & 0xff;
    g.order = key.to >> 8;
    dv3 s = ldd3(a.f.tx_pos + 3 * key.tx);
    g.R = ldd3(a.f.rx_pos + 3 * key.rx);
    g.P[0] = s;
#pragma unroll
    for (int j = 0; j < EMRT_KMAX; j++) g.tri[j] = -1;
    if (g.type == KT_LOS) {
        g.np = 2;
        return true;
    }
    if (g.type == KT_DIFF) {
        g.np = 3;
        g.w = wedge_of(S, key.ids[0]);
        return keller(g.w, s, g.R, a.diff_max_leg, g.P[1]);
    }
    if (g.type == KT_RD || g.type == KT_DR) {
        // one reflection unfolded by the image of Tx (reflection first) or of
        // Rx (diffraction first); the Keller point joins the real end to the
        // image, the reflection point is where the segment from the Keller
        // point to the image crosses the face plane
        const bool rd = g.type == KT_RD;
        const int f = rd ? key.ids[0] : key.ids[1];
        g.np = 4;
        g.w = wedge_of(S, rd ? key.ids[1] : key.ids[0]);
        if (f == g.w.f0 || f == g.w.fn) return false;
        const double* pl = S.plane + 4 * (long long)f;
        const dv3 img = rd ? mirror(s, pl) : mirror(g.R, pl);
        dv3 Q;
        if (!keller(g.w, rd ? img : s, rd ? g.R : img, a.diff_max_leg, Q)) return false;
        dv3 nrm = d3(pl[0], pl[1], pl[2]);
        dv3 dv = img - Q;
        double den = dot(nrm, dv);
        if (den == 0.0) return false;
        double tt = (pl[3] - dot(nrm, Q)) / den;
        if (!(tt > 0.0 && tt < 1.0)) return false;
        dv3 P = Q + dv * tt;
        int t = face_contains(a, f, P, stk);
        if (t < 0) return false;
        g.P[1] = rd ? P : Q;
        g.P[2] = rd ? Q : P;
        g.tri[rd ? 0 : 1] = t;
        return true;
    }
    const int order = g.order;
    g.np = order + 2;
    dv3 img[EMRT_KMAX + 1];
    img[0] = s;
#pragma unroll
    for (int i = 1; i <= EMRT_KMAX; i++)
        if (i <= order) img[i] = mirror(img[i - 1], S.plane + 4 * (long long)key.ids[i - 1]);
    dv3 cur = g.R;
#pragma unroll
    for (int i = EMRT_KMAX; i >= 1; i--) {
        if (i > order) continue;
        const double* pl = S.plane + 4 * (long long)key.ids[i - 1];
        dv3 nrm = d3(pl[0], pl[1], pl[2]);
        dv3 dv = img[i] - cur;
        double den = dot(nrm, dv);
        if (den == 0.0) return false;
        double tt = (pl[3] - dot(nrm, cur)) / den;
        if (!(tt > 0.0 && tt < 1.0)) return false;
        cur = cur + dv * tt;
        g.P[i] = cur;
        int t = face_contains(a, key.ids[i - 1], cur, stk);
        if (t < 0) return false;
        g.tri[i - 1] = t;
    }
    return true;
}

// endpoints and excluded faces of leg i (compile-time i)
template <int I>
__device__ __forceinline__ void leg_of(const Built& g, const KeyRec& key, dv3& p0, dv3& p1, int& xa, int& xb,
                                       int& xc) {
    p0 = g.P[I];
    p1 = (I + 2 == g.np) ? g.R : g.P[I + 1 <= EMRT_KMAX + 1 ? I + 1 : EMRT_KMAX + 1];
    xc = -1;
    if (g.type == KT_DIFF) {
        xa = g.w.f0;
        xb = g.w.fn;
    } else if (g.type == KT_RD || g.type == KT_DR) {
        // legs: Tx -> P -> Q -> Rx (RD) or Tx -> Q -> P -> Rx (DR); the faces
        // at a leg's ends are excluded: the reflection face at P, the two
        // wedge faces at Q
        const bool rd = g.type == KT_RD;
        const int f = rd ? key.ids[0] : key.ids[1];
        const bool p_at_start = rd ? I == 1 : I == 2, p_at_end = rd ? I == 0 : I == 1;
        const bool q_at_start = rd ? I == 2 : I == 1, q_at_end = rd ? I == 1 : I == 0;
        xa = (p_at_start || p_at_end) ? f : -1;
        xb = (q_at_start || q_at_end) ? g.w.f0 : -1;
        xc = (q_at_start || q_at_end) ? g.w.fn : -1;
    } else if (g.type == KT_SPEC) {
        xa = I >= 1 ? key.ids[I >= 1 ? I - 1 : 0] : -1;
        xb = I + 1 <= g.order ? key.ids[I < EMRT_KMAX ? I : EMRT_KMAX - 1] : -1;
    } else {
        xa = xb = -1;
    }
}

__device__ __forceinline__ KeyRec key_at(const PathArgs& a, long long q, long long n_links) {
    KeyRec key;
    if (q < n_links) {
        key.tx = (int)(q / a.f.n_rx);
        key.rx = (int)(q - (long long)key.tx * a.f.n_rx);
        key.to = KT_LOS;
#pragma unroll
        for (int j = 0; j < 5; j++) key.ids[j] = -1;
    } else {
        key = a.cand[q - n_links];
    }
    return key;
}

// shadow-ray record of leg I (compile-time) of a constructed key at slot pos
template <int I>
__device__ __forceinline__ void write_leg(const PathArgs& a, const Built& g, const KeyRec& key, unsigned long long pos,
                                          uint32_t q) {
    dv3 p0, p1;
    int xa, xb, xc;
    leg_of<I>(g, key, p0, p1, xa, xb, xc);
    dv3 d = p1 - p0;
    a.legs.ox[pos] = (float)p0.x; a.legs.oy[pos] = (float)p0.y; a.legs.oz[pos] = (float)p0.z;
    a.legs.dx[pos] = (float)d.x; a.legs.dy[pos] = (float)d.y; a.legs.dz[pos] = (float)d.z;
    a.legs.xa[pos] = xa;
    a.legs.xb[pos] = xb;
    a.legs.xc[pos] = xc;
    a.legs.key[pos] = q;
}

// Phase 1: exact construction of every key (line of sight for every link,
// then the candidates); surviving keys emit their legs as shadow rays.
__global__ void __launch_bounds__(128) k_construct(PathArgs a, long long n_links, long long cap_cand) {
    __shared__ int stk_lds[kStackDepth][kStackStride];  // columns of the first 128 threads used
    LdsStack stk{&stk_lds[0][threadIdx.x]};
    long long nc = (long long)*a.n_cand;
    if (nc > cap_cand) nc = cap_cand;
    long long n = n_links + nc;
    long long stride = (long long)gridDim.x * blockDim.x;
    long long start = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long iters = (n + stride - 1) / stride;
    for (long long it = 0; it < iters; it++) {
        long long q = start + it * stride;
        bool ok = q < n;
        KeyRec key;
        Built g;
        g.np = 0;
        if (ok) {
            key = key_at(a, q, n_links);
            ok = key_in_range(a, key) && construct(a, key, g, &stk);
            // state: 0 not constructed, 1 test every leg in full, 3 the
            // dynamic tree only (clear of the static scene, as at the last step)
            uint8_t stv = ok ? (uint8_t)1 : (uint8_t)0;
            uint32_t oc = 0u;
            if (ok && !a.moved_tx[key.tx] && !a.moved_rx[key.rx]) {
                if (q < n_links) {
                    if (a.los_sb[q]) oc = 1u;  // still blocked by the static scene
                    else stv = 3;
                } else if (a.cand_cached && key_static(a.s, key)) {
                    stv = 3;
                }
            }
            a.state[q] = stv;
            a.occl[q] = oc;
            if (ok) {
#pragma unroll
                for (int j = 0; j < EMRT_KMAX; j++) a.ktri[5 * q + j] = g.tri[j];
            }
        }
        // The leg that ends at the receiver takes slot q of the first region
        // [0, cap_first); the other legs go to [cap_first, cap), one
        // reservation per wave.  A key whose legs do not all fit is invalid,
        // but every reserved slot below the capacity is still written.
        const uint32_t nleg = ok ? (uint32_t)(g.np - 1) : 0u;
        const uint32_t n_other = nleg > 0u ? nleg - 1u : 0u;
        const unsigned long long po = wave_reserve(a.legs.count, n_other);
        const unsigned long long cap_f = (unsigned long long)a.legs.cap_first;
        const unsigned long long cap_o = (unsigned long long)(a.legs.cap - a.legs.cap_first);
        if (ok && po + n_other > cap_o) {
            atomicOr(a.flags, FLAG_PATH_CAP);
            a.state[q] = 0;
        }
        if (ok) {
            const uint32_t qq = (uint32_t)q;
            // slot of leg j, or ~0 when it falls beyond its region
            auto slot = [&](uint32_t j) -> unsigned long long {
                if (j + 1u == nleg) return (unsigned long long)q;
                return po + j < cap_o ? cap_f + po + j : ~0ULL;
            };
            unsigned long long s0 = slot(0), s1 = slot(1), s2 = slot(2), s3 = slot(3), s4 = slot(4), s5 = slot(5);
            if (s0 != ~0ULL) write_leg<0>(a, g, key, s0, qq);
            if (nleg > 1 && s1 != ~0ULL) write_leg<1>(a, g, key, s1, qq);
            if (nleg > 2 && s2 != ~0ULL) write_leg<2>(a, g, key, s2, qq);
            if (nleg > 3 && s3 != ~0ULL) write_leg<3>(a, g, key, s3, qq);
            if (nleg > 4 && s4 != ~0ULL) write_leg<4>(a, g, key, s4, qq);
            if (nleg > 5 && s5 != ~0ULL) write_leg<5>(a, g, key, s5, qq);
        }
    }
}

// Phase 2: float32 shadow rays over the open legs (t in (0, 1)), static and
// dynamic LBVH; a blocked leg marks its key occluded.  The leg that ends at
// the receiver goes first: it is the one most often blocked (the
// rays that proposed the key reached its first interaction, not the
// receiver), and a clear leg costs a full traversal where a blocked one stops
// at its first hit.  The other legs of the keys still open are then listed
// densely and traced.  Whether a key is occluded does not depend on the order
// of its legs.
// dyn_only: the leg is known clear of the static scene; los: a line of sight
// tested in full, whose static result is kept for the next step
__device__ __forceinline__ void shadow_leg(const PathArgs& a, long long i, uint32_t q, bool dyn_only, bool los,
                                           LdsStack* stk) {
    RayPre r = ray_pre(a.legs.ox[i], a.legs.oy[i], a.legs.oz[i], a.legs.dx[i], a.legs.dy[i], a.legs.dz[i]);
    int xa = a.legs.xa[i], xb = a.legs.xb[i], xc = a.legs.xc[i];
    bool hit = false;
    if (!dyn_only) {
        hit = any_hit4(a.st4, a.st, a.st_prims, r, 1.0f, xa, xb, xc, stk);
        if (los) a.los_sb[q] = hit ? 1 : 0;
    }
    if (hit || any_hit(a.dy, a.dy_prims, r, 1.0f, xa, xb, xc, stk)) a.occl[q] = 1u;
}

__global__ void __launch_bounds__(256) k_shadow_first(PathArgs a, long long n_links, long long cap_cand) {
    __shared__ int stk_lds[kStackRows][kStackStride];
    LdsStack stk{&stk_lds[0][threadIdx.x]};
    long long nc = (long long)*a.n_cand;
    if (nc > cap_cand) nc = cap_cand;
    GRID_STRIDE(q, n_links + nc) {
        const uint8_t stv = a.state[q];
        if (stv && !a.occl[q]) shadow_leg(a, q, (uint32_t)q, stv == 3, q < n_links, &stk);
    }
}

// The other legs of the keys still open, listed densely: a block takes
// kPickTile consecutive legs, counts its survivors, reserves their room with
// one atomic and writes them in leg order.
constexpr int kPickItems = 8;
constexpr long long kPickTile = 256LL * kPickItems;

__global__ void __launch_bounds__(256) k_shadow_pick(PathArgs a) {
    __shared__ uint32_t wcnt[4];
    __shared__ unsigned long long blk_base;
    const long long cap_o = a.legs.cap - a.legs.cap_first;
    long long n = (long long)*a.legs.count;
    if (n > cap_o) n = cap_o;
    const long long tile = (long long)blockIdx.x * kPickTile;
    if (tile >= n) return;  // the whole block
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    uint64_t m[kPickItems];
    uint32_t total = 0;
#pragma unroll
    for (int it = 0; it < kPickItems; it++) {
        long long j = tile + (long long)it * 256 + threadIdx.x;
        bool keep = j < n && !a.occl[a.legs.key[a.legs.cap_first + j]];
        m[it] = ballot64(keep);
        total += (uint32_t)__popcll(m[it]);
    }
    if (lane == 0) wcnt[w] = total;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        blk_base = t ? atomicAdd(a.legs.n_list, (unsigned long long)t) : 0ULL;
    }
    __syncthreads();
    unsigned long long base = blk_base;
    for (int v = 0; v < w; v++) base += wcnt[v];
#pragma unroll
    for (int it = 0; it < kPickItems; it++) {
        if ((m[it] >> lane) & 1ULL)
            a.legs.list[base + (unsigned long long)prefix_below(m[it])] =
                (uint32_t)(tile + (long long)it * 256 + threadIdx.x);
        base += (unsigned long long)__popcll(m[it]);
    }
}

__global__ void __launch_bounds__(256) k_shadow_rest(PathArgs a) {
    __shared__ int stk_lds[kStackRows][kStackStride];
    LdsStack stk{&stk_lds[0][threadIdx.x]};
    long long n = (long long)*a.legs.n_list;
    GRID_STRIDE(k, n) {
        long long i = a.legs.cap_first + (long long)a.legs.list[k];
        uint32_t q = a.legs.key[i];
        if (!a.occl[q]) shadow_leg(a, i, q, a.state[q] == 3, false, &stk);
    }
}

// Phase 3: fields of the unoccluded keys (double precision; the field model
// is in fields.h).  Delay L / c; Doppler (Section III-C, Eq (3) generalised
// to moving interaction points) -(1/lambda)[k_K.v_rx - k_0.v_tx +
// sum (k_{i-1} - k_i).v_obj]; AoD / AoA the directions of k_0 and -k_K.
// Survivors of the validation (constructed, no leg blocked) get their path
// slot from exclusive scans of 0/1 flags in key order, line of sight and
// specular paths first, then diffraction paths, so each field kernel runs on
// dense waves of one path type.
__global__ void __launch_bounds__(256) k_valid_flags(PathArgs a, long long n_links, long long cap_cand, ValidTemp t) {
    long long nc = (long long)*a.n_cand;
    if (nc > cap_cand) nc = cap_cand;
    long long n = n_links + nc;
    GRID_STRIDE(q, n) {  // the scans and the list read the first n flags only
        bool keep = a.state[q] && !a.occl[q];
        int type = keep && q >= n_links ? (a.cand[q - n_links].to & 0xff) : KT_LOS;
        bool r = keep && type >= KT_RD, d = keep && type == KT_DIFF;
        t.flag[q] = (keep && !d && !r) ? 1u : 0u;
        t.flag_d[q] = d ? 1u : 0u;
        t.flag_r[q] = r ? 1u : 0u;
    }
}

__global__ void __launch_bounds__(256) k_valid_list(ValidTemp t, const unsigned long long* n_cand, long long n_links,
                                                   long long cap_cand, unsigned long long* count) {
    const uint32_t n0 = t.cnt[0], n1 = t.cnt[1];
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = (unsigned long long)n0 + n1 + t.cnt[2];
    long long nc = (long long)*n_cand;
    if (nc > cap_cand) nc = cap_cand;
    GRID_STRIDE(q, n_links + nc) {
        if (t.flag[q]) t.surv[t.off[q]] = (uint32_t)q;
        else if (t.flag_d[q]) t.surv[n0 + t.off_d[q]] = (uint32_t)q;
        else if (t.flag_r[q]) t.surv[n0 + n1 + t.off_r[q]] = (uint32_t)q;
    }
}

// Fields of the survivors of one kind (KIND 1: line of sight and specular,
// 2: diffraction, 3: one reflection and one diffraction); the interaction points are rebuilt with the same formulas
// as the construction (image method / Keller point), the reflection
// triangles come from the construction.  Delay L / c; Doppler (Section
// III-C, Eq (3) generalised to moving interaction points) -(1/lambda)
// [k_K.v_rx - k_0.v_tx + sum (k_{i-1} - k_i).v_obj]; AoD / AoA the
// directions of k_0 and -k_K.
template <int KIND>
__global__ void __launch_bounds__(128) k_fields(PathArgs a, long long n_links, ValidTemp t) {
    const long long c0 = t.cnt[0], c1 = c0 + t.cnt[1], c2 = c1 + t.cnt[2];
    const long long lo = KIND == 1 ? 0 : (KIND == 2 ? c0 : c1);
    const long long hi = KIND == 1 ? c0 : (KIND == 2 ? c1 : c2);
    const SceneDev& S = a.s;
    // diffraction: one thread per (path, carrier), whose UTD coefficients are
    // the long part; the geometry is recomputed by each of them
    const int split = KIND == 2 ? a.fc.nf : 1;
    for (long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x; it < (hi - lo) * split;
         it += (long long)gridDim.x * blockDim.x) {
        const long long pos = lo + it / split;
        const int f0 = (int)(it - (pos - lo) * split);
        FieldCtx fc = a.fc;
        if (split > 1) {
            fc.nf = 1;
            fc.freq[0] = a.fc.freq[f0];
        }
        long long q = t.surv[pos];
        KeyRec key = key_at(a, q, n_links);
        dv3 sx = ldd3(a.f.tx_pos + 3 * key.tx), rx = ldd3(a.f.rx_pos + 3 * key.rx);
        PathGeo<double> pg;
        path_points<double, KIND>(S, key, v3c<double>(sx), rx, pg);
        dv3 vt = ldd3(a.f.tx_vel + 3 * key.tx), vr = ldd3(a.f.rx_vel + 3 * key.rx);
        double th = a.f.tx_orient[2 * key.tx], phi = a.f.tx_orient[2 * key.tx + 1];
        V3<double> kk[EMRT_KMAX + 1];
        double L;
        Cx<double> amp[EMRT_NF];
        path_field<double, KIND>(S, fc, key, pg, th, phi, 0, kk, L, amp);
        const int nlegs = pg.np - 1;
        constexpr int kLegs = KIND == 2 ? 2 : (KIND == 3 ? 3 : EMRT_KMAX + 1);  // at most, for this kind
        dv3 k0 = val3(kk[0]);
        dv3 kK = k0;
#pragma unroll
        for (int i = 1; i < kLegs; i++)
            if (i == nlegs - 1) kK = val3(kk[i]);
        double dop = dot(kK, vr) - dot(k0, vt);
        if (KIND == 1) {
#pragma unroll
            for (int i = 1; i <= EMRT_KMAX; i++) {
                if (i > pg.order || pg.type != KT_SPEC) break;
                int od = S.face_dyn[key.ids[i - 1]];
                if (od >= 0) dop += dot(val3(kk[i - 1]) - val3(kk[i]), ldd3(a.f.obj_vel + 3 * (long long)od));
            }
        } else {
            // the edge at Q and, for one reflection with the diffraction, the face at P
            const bool rd = pg.type == KT_RD, dr = pg.type == KT_DR;
            const int iq = rd ? 1 : 0;
            int od = S.face_dyn[S.edge_i[6 * (long long)(rd ? key.ids[1] : key.ids[0]) + 2]];
            if (od >= 0) dop += dot(val3(kk[iq]) - val3(kk[iq + 1]), ldd3(a.f.obj_vel + 3 * (long long)od));
            if (rd || dr) {
                const int ip = rd ? 1 : 2;  // legs ip - 1 and ip meet at P
                int of = S.face_dyn[rd ? key.ids[0] : key.ids[1]];
                if (of >= 0) dop += dot(val3(kk[ip - 1]) - val3(kk[ip]), ldd3(a.f.obj_vel + 3 * (long long)of));
            }
        }
        ValidPaths& o = a.out;
        const int nf_here = KIND == 2 ? 1 : fc.nf;  // KIND 2: this thread's carrier only
        for (int j = 0; j < nf_here; j++) {
            const int fi = j + (split > 1 ? f0 : 0);
            double lam = kC0 / a.fc.freq[fi];
            o.a[2 * (pos * a.fc.nf + fi)] = amp[j].re;
            o.a[2 * (pos * a.fc.nf + fi) + 1] = amp[j].im;
            o.fd[pos * a.fc.nf + fi] = -dop / lam;
        }
        if (f0 != 0) continue;
        o.key[pos] = key;
#pragma unroll
        for (int j = 0; j < 5; j++)
            o.tri[5 * pos + j] = (pg.type == KT_SPEC || pg.type >= KT_RD) ? a.ktri[5 * q + j] : -1;
        o.tau[pos] = L / kC0;
        float aod_az = (float)atan2(k0.y, k0.x), aod_el = (float)asin(fmin(1.0, fmax(-1.0, k0.z)));
        float aoa_az = (float)atan2(-kK.y, -kK.x), aoa_el = (float)asin(fmin(1.0, fmax(-1.0, -kK.z)));
        o.ang[pos] = make_float4(aod_az, aod_el, aoa_az, aoa_el);
    }
}

void validate_eval(const PathArgs& a, long long n_links, long long cap_cand, const ValidTemp& t, hipStream_t st) {
    long long n = n_links + cap_cand;
    hipLaunchKernelGGL(k_construct, dim3(grid_for(n, 128, 16384)), dim3(128), 0, st, a, n_links, cap_cand);
    hipLaunchKernelGGL(k_shadow_first, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, a, n_links, cap_cand);
    const long long cap_o = a.legs.cap - a.legs.cap_first;
    hipLaunchKernelGGL(k_shadow_pick, dim3((unsigned)((cap_o + kPickTile - 1) / kPickTile)), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_shadow_rest, dim3(grid_for(a.legs.cap, 256, 16384)), dim3(256), 0, st, a);
    int g = grid_for(n, 256, 16384);
    hipLaunchKernelGGL(k_valid_flags, dim3(g), dim3(256), 0, st, a, n_links, cap_cand, t);
    exclusive_scan_dev(t.flag, t.off, a.n_cand, n_links, n, t.scan_tmp, t.cnt, st);
    exclusive_scan_dev(t.flag_d, t.off_d, a.n_cand, n_links, n, t.scan_tmp, t.cnt + 1, st);
    if (a.combined) exclusive_scan_dev(t.flag_r, t.off_r, a.n_cand, n_links, n, t.scan_tmp, t.cnt + 2, st);
    else fill_u32(t.cnt + 2, 0u, 1, st);  // no combined keys pass key_in_range
    hipLaunchKernelGGL(k_valid_list, dim3(g), dim3(256), 0, st, t, a.n_cand, n_links, cap_cand, a.out.count);
    hipLaunchKernelGGL(k_fields<1>, dim3(grid_for(n, 128, 16384)), dim3(128), 0, st, a, n_links, t);
    hipLaunchKernelGGL(k_fields<2>, dim3(grid_for(n, 128, 16384)), dim3(128), 0, st, a, n_links, t);
    if (a.combined)
        hipLaunchKernelGGL(k_fields<3>, dim3(grid_for(n, 128, 16384)), dim3(128), 0, st, a, n_links, t);
}

// ----------------------------------------------------------- per link ----
// Key order within each link, in parallel: every valid path counts the paths
// of its link whose key sorts before its own and moves to that rank (equal
// keys, which a deduplicated path set does not hold, would keep their
// positions' order), so the link's later sums run in key order whatever order
// validation produced them in.
__global__ void k_link_rank(ValidPaths vp, int n_rx, const uint32_t* in, const int* start, const int* end,
                            uint32_t* out) {
    long long n = (long long)*vp.count;
    if (n > vp.cap) n = vp.cap;
    GRID_STRIDE(i, n) {
        uint32_t v = in[i];
        KeyRec kv = vp.key[v];
        long long L = (long long)kv.tx * n_rx + kv.rx;
        int s = start[L], e = end[L];
        int r = 0;
        for (int j = s; j < e; j++) {
            if (j == (int)i) continue;
            KeyRec kj = vp.key[in[j]];
            r += (key_less(kj, kv) || (j < (int)i && !key_less(kv, kj))) ? 1 : 0;
        }
        out[s + r] = v;
    }
}

void link_rank(const ValidPaths& vp, int n_rx, const uint32_t* in, const int* start, const int* end, uint32_t* out,
               hipStream_t st) {
    hipLaunchKernelGGL(k_link_rank, dim3(grid_for(vp.cap)), dim3(256), 0, st, vp, n_rx, in, start, end, out);
}

// Valid paths grouped by link with a counting sort: per-link counts
// (atomics on scattered addresses), an exclusive scan, then each path takes
// the next slot of its link.  The order inside a link is then arbitrary;
// k_link_rank puts it in key order.
__global__ void k_link_count(ValidPaths vp, int n_rx, uint32_t* cnt) {
    long long n = (long long)*vp.count;
    if (n > vp.cap) n = vp.cap;
    GRID_STRIDE(i, n) {
        KeyRec k = vp.key[i];
        atomicAdd(&cnt[(long long)k.tx * n_rx + k.rx], 1u);
    }
}

// start / end of every link's run (start -1 when empty); cnt becomes the
// scatter cursor (the run's start)
__global__ void k_link_bounds(uint32_t* cnt, const uint32_t* off, int* start, int* end, long long n_links) {
    GRID_STRIDE(L, n_links) {
        uint32_t c = cnt[L], o = off[L];
        start[L] = c ? (int)o : -1;
        end[L] = (int)(o + c);
        cnt[L] = o;
    }
}

__global__ void k_link_scatter(ValidPaths vp, int n_rx, uint32_t* cursor, uint32_t* order) {
    long long n = (long long)*vp.count;
    if (n > vp.cap) n = vp.cap;
    GRID_STRIDE(i, n) {
        KeyRec k = vp.key[i];
        order[atomicAdd(&cursor[(long long)k.tx * n_rx + k.rx], 1u)] = (uint32_t)i;
    }
}

void link_group(const ValidPaths& vp, int n_rx, long long n_links, uint32_t* cnt, uint32_t* off, uint32_t* scan_tmp,
                int* start, int* end, uint32_t* order, hipStream_t st) {
    fill_u32(cnt, 0u, n_links, st);
    hipLaunchKernelGGL(k_link_count, dim3(grid_for(vp.cap)), dim3(256), 0, st, vp, n_rx, cnt);
    exclusive_scan(cnt, off, n_links, scan_tmp, nullptr, st);
    hipLaunchKernelGGL(k_link_bounds, dim3(grid_for(n_links)), dim3(256), 0, st, cnt, off, start, end, n_links);
    hipLaunchKernelGGL(k_link_scatter, dim3(grid_for(vp.cap)), dim3(256), 0, st, vp, n_rx, cnt, order);
}

// One thread per link, over the link's paths in key order (the sums then run
// in a fixed order, so results are bit-reproducible):
//   H = sum a, P_coh = P_tx |H|^2, P_inc = P_tx sum |a|^2,
//   power-weighted mean and RMS of delay and Doppler (weights |a|^2).
// chan[(f * n_links + link) * 8 + {H.re, H.im, P_coh, P_inc, tau_mean,
// tau_rms, fd_mean, fd_rms}]; chan_i[link * 2 + {n_paths, los}].
__global__ void k_link_reduce(ValidPaths vp, const uint32_t* order, const int* start, const int* end,
                              long long n_links, int nf, double p_tx, double* chan, int* chan_i) {
    GRID_STRIDE(Lk, n_links) {
        int s = start[Lk], e = end[Lk];
        if (s < 0) {
            for (int f = 0; f < nf; f++)
                for (int c = 0; c < 8; c++) chan[((long long)f * n_links + Lk) * 8 + c] = 0.0;
            chan_i[2 * Lk] = 0;
            chan_i[2 * Lk + 1] = 0;
            continue;
        }
        int los = (vp.key[order[s]].to & 0xff) == KT_LOS ? 1 : 0;
        for (int f = 0; f < nf; f++) {
            double hr = 0, hi = 0, sw = 0, st_ = 0, sf = 0;
            for (int i = s; i < e; i++) {
                long long p = order[i];
                double ar = vp.a[2 * (p * nf + f)], ai = vp.a[2 * (p * nf + f) + 1];
                double wgt = ar * ar + ai * ai;
                hr += ar;
                hi += ai;
                sw += wgt;
                st_ += wgt * vp.tau[p];
                sf += wgt * vp.fd[p * nf + f];
            }
            double tm = sw > 0 ? st_ / sw : 0.0, fm = sw > 0 ? sf / sw : 0.0;
            double vt = 0, vf = 0;
            for (int i = s; i < e; i++) {
                long long p = order[i];
                double ar = vp.a[2 * (p * nf + f)], ai = vp.a[2 * (p * nf + f) + 1];
                double wgt = ar * ar + ai * ai;
                double dt = vp.tau[p] - tm, df = vp.fd[p * nf + f] - fm;
                vt += wgt * dt * dt;
                vf += wgt * df * df;
            }
            double* c = chan + ((long long)f * n_links + Lk) * 8;
            c[0] = hr;
            c[1] = hi;
            c[2] = p_tx * (hr * hr + hi * hi);
            c[3] = p_tx * sw;
            c[4] = tm;
            c[5] = sw > 0 ? sqrt(vt / sw) : 0.0;
            c[6] = fm;
            c[7] = sw > 0 ? sqrt(vf / sw) : 0.0;
        }
        chan_i[2 * Lk] = e - s;
        chan_i[2 * Lk + 1] = los;
    }
}

void link_reduce(const ValidPaths& vp, const uint32_t* order, const int* start, const int* end, long long n_links, int nf,
                 double p_tx, double* chan, hipStream_t st) {
    int* chan_i = (int*)(chan + (long long)nf * n_links * 8);
    hipLaunchKernelGGL(k_link_reduce, dim3(grid_for(n_links, 128)), dim3(128), 0, st, vp, order, start, end, n_links,
                       nf, p_tx, chan, chan_i);
}

__global__ void k_cache_counts(ValidPaths vp, const uint32_t* order, const int* start, const int* end,
                               long long n_links, uint32_t* per_link) {
    GRID_STRIDE(Lk, n_links) {
        int s = start[Lk], e = end[Lk];
        uint32_t c = 0;
        if (s >= 0) {
            c = (uint32_t)(e - s);
            if ((vp.key[order[s]].to & 0xff) == KT_LOS) c--;
        }
        per_link[Lk] = c;
    }
}

void cache_counts(const ValidPaths& vp, const uint32_t* order, const int* start, const int* end, long long n_links,
                  uint32_t* per_link, hipStream_t st) {
    hipLaunchKernelGGL(k_cache_counts, dim3(grid_for(n_links)), dim3(256), 0, st, vp, order, start, end, n_links,
                       per_link);
}

__global__ void k_cache_write(ValidPaths vp, const uint32_t* order, const int* start, const int* end,
                              const uint32_t* off, long long n_links, KeyRec* cache) {
    GRID_STRIDE(Lk, n_links) {
        int s = start[Lk], e = end[Lk];
        if (s < 0) continue;
        uint32_t o = off[Lk];
        for (int i = s; i < e; i++) {
            KeyRec k = vp.key[order[i]];
            if ((k.to & 0xff) == KT_LOS) continue;
            cache[o++] = k;
        }
    }
}

void cache_write(const ValidPaths& vp, const uint32_t* order, const int* start, const int* end, const uint32_t* off,
                 long long n_links, KeyRec* cache, hipStream_t st) {
    hipLaunchKernelGGL(k_cache_write, dim3(grid_for(n_links)), dim3(256), 0, st, vp, order, start, end, off, n_links,
                       cache);
}

__global__ void k_path_gather(ValidPaths vp, const uint32_t* order, const int* start, const int* end,
                              long long n_links, int nf, int cap, int32_t* key, int32_t* tri, double* a, double* tau,
                              double* fd, float* ang, int32_t* count) {
    GRID_STRIDE(Lk, n_links) {
        int s = start[Lk], e = end[Lk];
        int n = s < 0 ? 0 : e - s;
        int m = n < cap ? n : cap;
        if (count) count[Lk] = m;
        for (int j = 0; j < m; j++) {
            long long p = order[s + j];
            long long o = Lk * cap + j;
            KeyRec k = vp.key[p];
            if (key) {
                int32_t* kr = key + 9 * o;
                kr[0] = k.tx; kr[1] = k.rx; kr[2] = k.to & 0xff; kr[3] = k.to >> 8;
                for (int q = 0; q < 5; q++) kr[4 + q] = k.ids[q];
            }
            if (tri) for (int q = 0; q < 5; q++) tri[5 * o + q] = vp.tri[5 * p + q];
            if (a) for (int f = 0; f < nf; f++) {
                a[2 * (o * nf + f)] = vp.a[2 * (p * nf + f)];
                a[2 * (o * nf + f) + 1] = vp.a[2 * (p * nf + f) + 1];
            }
            if (tau) tau[o] = vp.tau[p];
            if (fd) for (int f = 0; f < nf; f++) fd[o * nf + f] = vp.fd[p * nf + f];
            if (ang) {
                float4 g = vp.ang[p];
                ang[4 * o] = g.x; ang[4 * o + 1] = g.y; ang[4 * o + 2] = g.z; ang[4 * o + 3] = g.w;
            }
        }
    }
}

void path_gather(const ValidPaths& vp, const uint32_t* order, const int* start, const int* end, long long n_links,
                 int nf, int cap, int32_t* key, int32_t* tri, double* a, double* tau, double* fd, float* ang,
                 int32_t* count, hipStream_t st) {
    hipLaunchKernelGGL(k_path_gather, dim3(grid_for(n_links)), dim3(256), 0, st, vp, order, start, end, n_links, nf,
                       cap, key, tri, a, tau, fd, ang, count);
}

__global__ void k_keys_export(const KeyRec* c, long long n, int32_t* out) {
    GRID_STRIDE(i, n) {
        KeyRec k = c[i];
        int32_t* r = out + 9 * i;
        r[0] = k.tx; r[1] = k.rx; r[2] = k.to & 0xff; r[3] = k.to >> 8;
        for (int q = 0; q < 5; q++) r[4 + q] = k.ids[q];
    }
}

__global__ void k_keys_import(const int32_t* in, long long n, KeyRec* c) {
    GRID_STRIDE(i, n) {
        const int32_t* r = in + 9 * i;
        KeyRec k;
        k.tx = r[0]; k.rx = r[1]; k.to = r[2] | (r[3] << 8);
        for (int q = 0; q < 5; q++) k.ids[q] = r[4 + q];
        c[i] = k;
    }
}

void keys_export(const KeyRec* cache, long long n, int32_t* out, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_keys_export, dim3(grid_for(n)), dim3(256), 0, st, cache, n, out);
}
void keys_import(const int32_t* in, long long n, KeyRec* cache, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_keys_import, dim3(grid_for(n)), dim3(256), 0, st, in, n, cache);
}

}  // namespace emrt
