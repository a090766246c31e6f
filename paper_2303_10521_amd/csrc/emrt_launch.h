// emrt_launch.h -- host-side launch interface between the library's
// translation units (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "emrt_dev.h"

namespace emrt {

// ------------------------------------------------------------ sort.hip ----
size_t scan_temp_bytes(long long n);
void exclusive_scan(const uint32_t* in, uint32_t* out, long long n, uint32_t* temp, uint32_t* grand, hipStream_t st);
// over the first min(*n_dev + add, cap) values (a device-side count); temp as for a scan of cap values
void exclusive_scan_dev(const uint32_t* in, uint32_t* out, const unsigned long long* n_dev, long long add,
                        long long cap, uint32_t* temp, uint32_t* grand, hipStream_t st);
size_t radix_temp_bytes(long long cap);
int radix_sort(unsigned long long* k0, uint32_t* v0, unsigned long long* k1, uint32_t* v1, const long long* n_dev,
               long long cap, int nbits, void* temp, hipStream_t st);
void fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t st);
void fill_u64(unsigned long long* p, unsigned long long v, long long n, hipStream_t st);
void iota_u32(uint32_t* p, long long n, hipStream_t st);

// ------------------------------------------------------------- bvh.hip ----
// A binary LBVH over n primitives given as float boxes [n][6] (lo, hi).
struct Tree {
    BNode* nodes = nullptr;       // [max(n-1, 1)]
    int* leaf_parent = nullptr;   // [n] parent | side << 31
    uint32_t* counters = nullptr; // [max(n-1, 1)] refit arrival counters
    uint32_t* perm = nullptr;     // [n] leaf slot -> primitive index
    int* span = nullptr;          // [max(n-1, 1)] LBVH: the far end of node i's leaf range (i is the other)
    bool lbvh = false;            // built by bvh_build_many (span valid)
    int n = 0;
    int cap = 0;
    Bvh view() const { return Bvh{nodes, n}; }
};
// scratch for a build of up to `cap` primitives
struct BuildTemp {
    unsigned long long* k0;
    unsigned long long* k1;
    uint32_t* v0;
    uint32_t* v1;
    uint32_t* bounds;  // [64]
    void* radix;
};
size_t build_temp_bytes(long long cap);
void carve_build_temp(void* base, long long cap, BuildTemp& t);
void bvh_build(const float* box6, int n, Tree& tree, const BuildTemp& tmp, hipStream_t st);
// up to kMaxBuildJobs trees in one batch (one sort, one launch per later stage);
// `tmp` must hold the sum of their primitive counts
constexpr int kMaxBuildJobs = 4;
struct BuildJob {
    const float* box6;
    int n;
    Tree* tree;
};
void bvh_build_many(const BuildJob* jobs, int n_jobs, const BuildTemp& tmp, hipStream_t st);
void bvh_refit(const float* box6, Tree& tree, hipStream_t st);
// out2 (device, 2 doubles): summed child box areas over all nodes, root box area
void tree_quality(const Tree& tree, double* out2, hipStream_t st);
// top-down binned SAH build into the same node format (static scene, once): one launch per level,
// synchronises per level; returns the number of levels, -1 on a HIP error
int bvh_build_sah(const float* box6, int n, Tree& tree, const BuildTemp& tmp, hipStream_t st);
// extra tree statistics: surface-area sum of internal nodes (device double)
void bvh_sah(const Tree& tree, double* out, hipStream_t st);
// Host: collapse a binary tree (its internal nodes read back from the device,
// root first) into 4-wide nodes with quantised child boxes (QNode4), root
// first, parents before children.  Returns the node count.
int bvh4_collapse(const BNode* bin, int n_prims, QNode4* out, int cap);

// ----------------------------------------------------------- scene.hip ----
struct SceneDev {
    int V, T, F, O, M;
    const float* verts_local;   // [V][3] caller's array, copied at set_scene
    float* verts_local_copy;    // [V][3]
    float* verts;               // [V][3] world vertices of the current frame
    int* tris;                  // [T][3]
    int* tri_face;              // [T]
    int* face_object;           // [F]
    int* face_material;         // [F]
    int* face_dyn;              // [F] dynamic-object rank or -1
    int* vert_dyn;              // [V]
    int* obj_rank;              // [O] dynamic rank or -1
    double* plane;              // [F][4]
    int* face_first;            // [F] lowest triangle id
    int* face_off;              // [F+1]
    int* face_tris;             // [T] sorted by (face, tri)
    float* face_tv;             // [T][9] world vertices of face_tris[q] (refreshed every frame)
    float* face_box;            // [F][6] bounding box (lo, hi) of each face (refreshed every frame)
    int* tris_static;           // [T_s]
    int* tris_dynamic;          // [T_d]
    int T_s, T_d, O_d;
    // wedge edges
    int E, E_cap;
    int* edge_i;                // [E][6] va, vb, f0, fn, w0, wn
    double* edge_n;             // [E]
    int* edges_static;          // [E_s] ids of the edges of static objects, in edge order
    int* edges_dynamic;         // [E_dyn] ids of the edges of moving objects, in edge order
    int E_s, E_dyn;
};

// validate indices; returns flags via device word
void scene_check(const SceneDev& s, const uint8_t* object_dynamic, uint32_t* flags, hipStream_t st);
void scene_prepare(SceneDev& s, const uint8_t* object_dynamic, uint32_t* scratch_u32, int* counts_dev,
                   const BuildTemp& tmp, hipStream_t st);
int scene_edges(SceneDev& s, int* obj_off, int* obj_faces, int* counter, const BuildTemp& tmp, hipStream_t st);
void scene_world(const SceneDev& s, const double* xform, uint32_t* flags, hipStream_t st);
void scene_planes(const SceneDev& s, hipStream_t st);
// face-ordered triangle vertices (face_tv) of the current world vertices
void scene_face_tv(const SceneDev& s, hipStream_t st);
void tri_boxes(const SceneDev& s, const int* list, int n, float* box6, hipStream_t st);
void tri_prims(const SceneDev& s, const int* list, const Tree& tree, TriP* prims, hipStream_t st);
void edge_boxes(const SceneDev& s, const int* list, int n, float* box6, hipStream_t st);
// Splits the wedge edges into those of static and of moving objects
// (s.edges_static / s.edges_dynamic, s.E_s / s.E_dyn).  scratch: 2 E + 16
// u32 and a scan temp of E; count_dev: one device int.  Returns E_s, or -1 on
// a HIP error (synchronises the stream).
int edge_partition(SceneDev& s, uint32_t* scratch, int* count_dev, hipStream_t st);
// boxes / leaf primitives of the edges list[0, n) (prims by the tree's leaf
// order; each primitive carries its edge id)
void edge_prims(const SceneDev& s, const int* list, const Tree& tree, float4* prims, hipStream_t st);
void rx_boxes(const double* rx_pos, int n_rx, float* box6, hipStream_t st);
void rx_prims(const double* rx_pos, const Tree& tree, float4* prims, hipStream_t st);

// ----------------------------------------------------------- trace.hip ----
struct RaySoA {
    float *ox, *oy, *oz, *dx, *dy, *dz, *L;
    uint32_t* id;
    int* prev;
};

struct BounceArgs {
    RaySoA in, out;
    const unsigned long long* n_in;
    unsigned long long* n_out;
    // regroup key of every surviving ray (null: none): its origin's cell on a
    // 16 x 16 grid over the scene's x, y extent (cell = (x - key_ox) key_sx)
    // in Morton order, then its direction octant
    uint16_t* out_key;
    float key_ox, key_oy, key_sx, key_sy;
    unsigned int* work;
    int b, K;
    long long n_total;
    int rays_per_tx;
    // scene
    Bvh st, dy;
    Bvh4 st4;  // the static tree collapsed to 4-wide quantised nodes (same leaves as st)
    const TriP* st_prims;
    const TriP* dy_prims;
    const double* plane;
    // receivers
    Bvh rxt;
    const float4* rx_prims;
    float alpha_k;  // k_rx * sqrt(4 pi / N)
    float4 rx_root_lo, rx_root_hi;  // unused when the tree is read on device
    // edges
    int diffraction;
    Bvh ets, etd;                               // edges of static objects (built once) and of moving ones
    const float4 *eprims_s, *eprims_d;          // their leaf primitives, [E_s][2] and [E_dyn][2]
    uint32_t* illum;           // [N_tx][E_words]
    int e_words;
    unsigned long long* pairs; // (source, face, edge) lit by second segments (diffraction = 2)
    unsigned long long pair_mask;
    // path table
    unsigned long long* table;
    unsigned long long mask;
    KeySrc src;
    int* hitlog;
    uint8_t* depth;             // [n_total] the bounce at which each ray ended (hit log rows beyond it are stale)
    uint32_t* flags;
    unsigned long long* stats;  // [4] node visits, triangle tests, segments, captures (STATS only)
    // bounce 0 of a transmitter-side launch makes its rays itself: ray k leaves
    // source k / gen_N along gen_dirs[k % gen_N] (null: read `in`)
    const float4* gen_dirs;
    const double* gen_src;
    int gen_N;
    // capture log of marked rays (transmitter-side discovery; null: off):
    // rows (launch slot, bounce | kind << 8, receiver or edge)
    const uint32_t* dbg_sel;  // [n_total / 32 + 1] mark bit per launch slot
    int* dbg_log;             // [dbg_cap][3]
    unsigned long long* dbg_n;
    long long dbg_cap;
};
void ray_order(int N, uint32_t* perm, const BuildTemp& tmp, hipStream_t st);
// the N launch directions in launch order (perm: direction index of each slot)
void dir_table(const uint32_t* perm, int N, float4* dirs, hipStream_t st);
// sources src_pos [n_src][3], N directions each; perm: launch order of the directions (null: index order)
void raygen(const double* src_pos, int n_src, int N, const uint32_t* perm, RaySoA out, unsigned long long* n_out,
            hipStream_t st);
void bounce(const BounceArgs& a, bool stats, int grid, hipStream_t st);
// Regrouping of the rays between bounces: constants and workspace.
constexpr int kRegroupBins = 2048;  // 256 origin cells x 8 direction octants
int regroup_blocks(long long n_total);
size_t regroup_temp_u32(long long n_total);  // u32 of per-block histograms, their offsets and the scan temp
// Rays [0, *n_dev) of src into dst, grouped by key (one counting sort: per-block
// histograms in LDS, an exclusive scan, a scatter); within a key the blocks'
// ranges keep their order.  temp: regroup_temp_u32(cap) u32.
void regroup(const RaySoA& src, const RaySoA& dst, const uint16_t* key, const unsigned long long* n_dev, long long cap,
             uint32_t* temp, hipStream_t st);
// one launch over several scenes' live rays (args device [n_scenes]; chunk_off [n_scenes + 1], work: scratch)
void bounce_multi(const BounceArgs* args, int n_scenes, uint32_t* chunk_off, uint32_t* work, int grid, int chunk,
                  hipStream_t st);
void debug_rays(const int* hitlog, const uint8_t* depth, long long n_total, int K, int tx, int N,
                const uint32_t* slot_of, const int* ray_ids, int n, int* out, hipStream_t st);
// mark the launch slots of directions ray_ids of transmitter tx (bad: set when one is out of range)
void debug_mark(uint32_t* sel, int tx, int N, const uint32_t* slot_of, const int* ray_ids, int n, uint32_t* bad,
                hipStream_t st);
// log rows -> (tx, direction, bounce, kind, id) through the launch order perm (direction of each slot)
void debug_captures(const int* log, const unsigned long long* n_log, long long log_cap, int N, const uint32_t* perm,
                    int* out, long long cap, hipStream_t st);
// inv[perm[t]] = t
void invert_perm(const uint32_t* perm, uint32_t* inv, int n, hipStream_t st);

// ----------------------------------------------------------- paths.hip ----
struct FrameDev {
    int n_tx, n_rx;
    const double* tx_pos;   // [N_tx][3]
    const double* tx_vel;
    const double* tx_orient;  // [N_tx][2]
    const double* rx_pos;
    const double* rx_vel;
    const double* obj_vel;  // [O_d][3]
};

struct ValidPaths {
    KeyRec* key;
    int* tri;        // [cap][5]
    double* a;       // [cap][nf][2]
    double* tau;     // [cap]
    double* fd;      // [cap][nf]
    float4* ang;     // [cap]
    unsigned long long* count;
    long long cap;
};

// shadow rays of the keys under validation (one per leg)
struct LegBuf {
    float *ox, *oy, *oz, *dx, *dy, *dz;
    int *xa, *xb, *xc;  // faces excluded from the leg's shadow ray
    uint32_t* key;      // key slot
    // [0, cap_first): slot q holds the leg of key q that ends at the
    // receiver; [cap_first, cap): the keys' other legs (*count of them)
    unsigned long long* count;
    long long cap_first;
    long long cap;
    uint32_t* list;     // [cap - cap_first] other legs still to trace (*n_list)
    unsigned long long* n_list;
};

// inputs of the field evaluation shared by the forward and the adjoint
struct FieldCtx {
    const double* mat_eps;  // [M][2] relative permittivities
    const double* mat_refl; // [M] 0: Fresnel from mat_eps; g > 0: constant reflection coefficient magnitude
    double freq[EMRT_NF];   // carriers, Hz
    int nf;
    int ant_mode;           // transmit antenna
};

struct PathArgs {
    SceneDev s;
    LegBuf legs;
    uint8_t* state;   // [n_links + cap_cand] 1 = constructed
    uint32_t* occl;   // [n_links + cap_cand] 1 = a leg is blocked
    int* ktri;        // [n_links + cap_cand][5] triangle of each reflection point of a constructed key
    FrameDev f;
    Bvh st, dy;
    Bvh4 st4;  // the static tree collapsed to 4-wide quantised nodes (same leaves as st)
    const TriP* st_prims;
    const TriP* dy_prims;
    FieldCtx fc;
    double diff_max_leg;
    int combined;     // one reflection with one diffraction in use (types 3 and 4 valid)
    // reuse of last step's tests against the static scene (the static tree never changes)
    const uint8_t* moved_tx;  // [n_tx] 1 = moved since the last step (or no last step)
    const uint8_t* moved_rx;  // [n_rx]
    uint8_t* los_sb;          // [n_links] 1 = line of sight blocked by the static scene at the last test
    int cand_cached;          // the candidates are last step's valid keys (a cached frame)
    // inputs
    const KeyRec* cand;
    const unsigned long long* n_cand;
    ValidPaths out;
    uint32_t* flags;
};

// moved[i] = position i differs from prev (or *hist == 0); prev := position
void endpoints_moved(const double* pos, double* prev, int n, uint8_t* moved, const uint32_t* hist, hipStream_t st);
void cache_insert(unsigned long long* table, unsigned long long mask, const KeyRec* cache,
                  const unsigned long long* n_cache, long long cap, KeySrc src, uint32_t* flags, hipStream_t st);
// receivers binned on a kGridN x kGridN grid over their x-y bounding box
constexpr int kGridN = 128;
struct RxGrid {
    float x0, y0, inv_h;  // cell (cx, cy) = floor((x - x0) inv_h), floor((y - y0) inv_h), clamped
};
struct RxBins {
    RxGrid* grid;
    uint32_t* cnt;       // [kGridN^2]
    uint32_t* cursor;    // [kGridN^2]
    uint32_t* start;     // [kGridN^2 + 1] first sorted receiver of each cell
    uint32_t* scan_tmp;
    float4* sorted;      // [n_rx] (x, y, z, receiver index) by cell
};
void rx_grid_build(const double* rx_pos, int n_rx, const RxBins& b, hipStream_t st);
// transmitter-side diffraction keys not in the cache, in the order they are made ([cap] u64 references)
struct FreshKeys {
    unsigned long long* ref;
    unsigned long long* count;
    long long cap;
};
void diff_candidates(const PathArgs& a, const uint32_t* illum, int e_words, const RxBins& bins,
                     const unsigned long long* table, unsigned long long mask, KeySrc src, const FreshKeys& fk,
                     hipStream_t st);
// the previous cache copied into cand[*n_cand, ...) and added to *n_cand (after the table's compaction,
// which leaves cache references out)
void cache_append(const KeyRec* cache, const unsigned long long* n_cache, long long cap_cache,
                  unsigned long long* n_cand, KeyRec* cand, long long cap, uint32_t* flags, hipStream_t st);
// the fresh keys expanded into cand[*n_cand, ...) and added to *n_cand (after the table's compaction)
void fresh_append(const FreshKeys& fk, unsigned long long* n_cand, KeyRec* cand, long long cap, KeySrc src,
                  uint32_t* flags, hipStream_t st);
// keys proposed outside the path table's own references (reflection-diffraction candidates)
struct ExtraKeys {
    KeyRec* key;
    unsigned long long* count;
    long long cap;
};
// (source, face, edge) pairs lit by second segments -> reflection-then-diffraction keys to the
// receivers near the edge (transmitter-side launch, src_rx null) or diffraction-then-reflection
// keys from every transmitter (receiver-side launch)
void pair_candidates(const PathArgs& a, const unsigned long long* set, long long n_slots, unsigned long long* list,
                     unsigned long long* n_list, const RxBins& bins, const int* src_rx, const ExtraKeys& xk,
                     unsigned long long* table, unsigned long long mask, KeySrc src, hipStream_t st);
// receiver-side launch: illum rows are the sources src_rx[0..n_src); every transmitter is tried
void diff_candidates_rx(const PathArgs& a, const uint32_t* illum, int e_words, const int* src_rx, int n_src,
                        unsigned long long* table, unsigned long long mask, KeySrc src, hipStream_t st);
void gather_rx(const double* rx_pos, const int* sel, int n, double* out, hipStream_t st);
// scratch of the table compaction: per-wave counts and offsets
// ([compact_temp_elems(n_slots)] each) + scan temp
struct CompactTemp {
    uint32_t* flags;
    uint32_t* off;
    uint32_t* scan_tmp;
};
long long compact_temp_elems(unsigned long long n_slots);
void table_compact(const unsigned long long* table, unsigned long long n_slots, KeySrc src, KeyRec* cand,
                   unsigned long long* n_cand, long long cap, uint32_t* flags, const CompactTemp& t, hipStream_t st);
// scratch of the validation: [n_links + cap_cand] survivor flags, offsets, list + scan temp
struct ValidTemp {
    uint32_t* flag;     // line of sight and specular survivors
    uint32_t* off;
    uint32_t* flag_d;   // diffraction survivors
    uint32_t* off_d;
    uint32_t* flag_r;   // survivors with one reflection and one diffraction
    uint32_t* off_r;
    uint32_t* cnt;      // [3] survivor counts of the three kinds
    uint32_t* surv;     // survivors, kind by kind
    uint32_t* scan_tmp;
};
void validate_eval(const PathArgs& a, long long n_links, long long cap_cand, const ValidTemp& t, hipStream_t st);
// valid paths grouped by link (order[start[L], end[L]) are link L's paths; start -1 when empty)
void link_group(const ValidPaths& vp, int n_rx, long long n_links, uint32_t* cnt, uint32_t* off, uint32_t* scan_tmp,
                int* start, int* end, uint32_t* order, hipStream_t st);
void link_rank(const ValidPaths& vp, int n_rx, const uint32_t* in, const int* start, const int* end, uint32_t* out,
               hipStream_t st);
void link_reduce(const ValidPaths& vp, const uint32_t* order, const int* start, const int* cnt, long long n_links, int nf,
                 double p_tx, double* chan, hipStream_t st);
void cache_counts(const ValidPaths& vp, const uint32_t* order, const int* start, const int* cnt, long long n_links,
                  uint32_t* per_link, hipStream_t st);
void cache_write(const ValidPaths& vp, const uint32_t* order, const int* start, const int* cnt, const uint32_t* off,
                 long long n_links, KeyRec* cache, hipStream_t st);
void path_gather(const ValidPaths& vp, const uint32_t* order, const int* start, const int* cnt, long long n_links,
                 int nf, int cap, int32_t* key, int32_t* tri, double* a, double* tau, double* fd, float* ang,
                 int32_t* count, hipStream_t st);
void keys_export(const KeyRec* cache, long long n, int32_t* out, hipStream_t st);
void keys_import(const int32_t* in, long long n, KeyRec* cache, hipStream_t st);

// -------------------------------------------------------- coherence.hip ----
#define EMRT_CORR_LAGS 4
struct CohState {
    unsigned long long* frames;  // steps since the last reset
    double* ring;                // [nf][n_links][EMRT_CORR_LAGS] last |H| values
    double* prod;                // [nf][n_links][EMRT_CORR_LAGS] sums of g_t g_{t-k}
    double* s1;                  // [nf][n_links] sum of g
    double* s2;                  // [nf][n_links] sum of g^2
    uint32_t* prev_los;          // [n_links]
    unsigned long long* prev_hash;  // [n_links] first-order key-set hash
    uint32_t* trigger;           // [n_links] bits of the last step
};
struct CohRead {
    double R;                    // correlation threshold of Eq (2)
    double* tc;                  // [nf][n_links] or null
    double* corr;                // [nf][n_links][EMRT_CORR_LAGS] or null
    uint32_t* trigger;           // [n_links] or null
    unsigned long long* min_tc;  // bit pattern of the smallest finite T_c (device), or null
    unsigned long long* n_triggered;
};
void coherence_update(const CohState& c, const ValidPaths& vp, const uint32_t* order, const int* start,
                      const int* end, const double* chan, long long n_links, int nf, hipStream_t st);
void coherence_read(const CohState& c, const CohRead& r, long long n_links, int n_rx, int nf, const double* tx_pos,
                    const double* tx_vel, const double* rx_pos, const double* rx_vel, const FieldCtx& fc,
                    hipStream_t st);

// ---------------------------------------------------------- adjoint.hip ----
struct AdjArgs {
    SceneDev s;
    FieldCtx fc;
    const double* tx_pos;     // [N_tx][3] frame of the last step
    const double* tx_orient;  // [N_tx][2]
    const double* rx_pos;     // [N_rx][3]
    ValidPaths vp;            // valid paths of the last step
    const uint32_t* order;    // path indices sorted by (link, key)
    const int* start;         // [n_links] first sorted index of a link, -1 if none
    const int* end;           // [n_links]
    const double* chan;       // channel sums of the last step (H at [(f n_links + l) 8 + 0, 1])
    const double* dL_dH;      // [nf][n_links][2] or null
    const double* dL_dP;      // [nf][n_links] or null
    double p_tx;
    long long n_links;
    int M;                    // materials
    int combined;             // paths with one reflection and one diffraction can occur
    double* rows;             // [5 + 2 M][n_links] per-link partial gradients
    int n_rx;
    double* path_tan;         // [vp.cap][5] per path: sum over carriers of Re(conj(g) da/dx), x = tx.xyz, theta, phi
    double* path_eps;         // [vp.cap][5][2] per path and interaction: g conj(da/deps) of its material
};
void adjoint(const AdjArgs& a, int n_tx, int n_rx, double* g_pos, double* g_ori, double* g_eps, hipStream_t st);

}  // namespace emrt
