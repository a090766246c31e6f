// api.hip -- the C ABI (include/emrt.h): context, workspace carving and the
// per-frame pipeline.  All device state lives in one caller-owned workspace;
// every launch goes to the context's stream and a frame needs no host round
// trip (element counts stay on the device).
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/emrt.h"
#include "emrt_dev.h"
#include "emrt_launch.h"

using namespace emrt;

namespace {

constexpr int kMaxMaterials = 256;
constexpr int kMaxRxSources = 1024;  // receivers of one receiver-side launch
constexpr int kNumCounters = 64;
// counter slots (u64)
constexpr int C_RAYS = 0;      // [0..7] live rays entering bounce b
constexpr int C_WORK = 8;      // [8..15] work counters per bounce
constexpr int C_NCAND = 16;
constexpr int C_NVALID = 17;
constexpr int C_NCACHE = 18;   // [18, 19] cache sizes (double buffer)
constexpr int C_STATS = 20;    // [20..23] and [36] (traversal counters)
constexpr int C_TRUNC = 24;    // path-list truncation flag
constexpr int C_NLEGS = 25;    // shadow legs of the step besides the receiver legs
constexpr int C_COH = 26;      // [26, 27] coherence read-back (min T_c bits, triggered links)
constexpr int C_NPAIRS = 28;   // listed (source, face, edge) pairs
constexpr int C_NEXTRA = 29;   // keys proposed into the extra-key array
constexpr int C_NFRESH = 30;   // transmitter-side diffraction keys not in the cache
constexpr int C_NLIST = 31;    // of those, the ones traced after the receiver legs
constexpr int C_SCRATCH = 32;  // ints for set_scene

struct Carver {
    char* base;
    size_t off = 0;
    bool measure;
    explicit Carver(char* b) : base(b), measure(b == nullptr) {}
    template <class T>
    T* take(long long n) {
        off = (off + 255) & ~(size_t)255;
        T* p = measure ? nullptr : (T*)(base + off);
        off += sizeof(T) * (size_t)(n > 0 ? n : 1);
        return p;
    }
};

int64_t pow2_at_least(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

struct emrt_ctx {
    emrt_config cfg{};
    emrt_sizes sz{};
    bool sized = false, bound = false, scene_set = false, frame_set = false, stepped = false, discovered = false;
    bool frame_since_step = false;  // set_frame after the last step (the adjoint needs the step's frame)
    bool batched = false;           // member of an emrt_batch
    double* adj_rows = nullptr;     // [5 + 2 adjoint_materials][n_links]
    char* leg_block = nullptr;      // shadow legs of a step; per-path partials of emrt_backward
    uint32_t* dbg_sel = nullptr;    // capture log: mark bit per launch slot
    int* dbg_log = nullptr;         // [EMRT_CAPTURE_LOG_ROWS][3]
    unsigned long long* dbg_n = nullptr;
    bool dbg_on = false;            // some ray is marked
    CompactTemp ctmp{};             // table compaction scratch
    RxBins bins{};                  // receivers binned for the diffraction candidates
    ValidTemp vtmp{};               // validation survivors
    int* ktri = nullptr;            // [vcap][5] reflection triangles of constructed keys
    CohState coh{};                 // coherence statistics over frames
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    // second stream of a single-context discovery step: the diffraction
    // candidates (they need only the first bounce) run beside bounces 1..K
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // quality of the moving objects' tree, read back one step late (the
    // rebuild-on-degradation policy): device pair, pinned copy, its event
    double* dyq_dev = nullptr;
    double* dyq_host = nullptr;
    hipEvent_t ev_dyq = nullptr;
    bool dyq_pending = false, dyq_pending_build = false;
    bool dy_updated = false, dy_updated_build = false;  // this step built or refitted the tree
    double dyq_built = 0.0, dyq_last = 0.0;
    int64_t dyn_rebuilds = 0;
    bool diff_async = false;
    std::string err;
    int stats_on = 0, timing_on = 0;
    // kernel timing: two event sets used by alternate steps, read lazily so
    // consecutive steps never wait for each other
    struct EventSet {
        hipEvent_t ev[16];
        int used = 0, bounce_end = 0;
        bool pending = false;
    } evs[2];
    bool ev_created = false;
    int ev_parity = 0;
    double t_bounce_ms = 0, t_validate_ms = 0;
    int t_bounce_n = 0, t_validate_n = 0;

    // derived sizes
    long long n_total = 0, n_links = 0, P = 0, table_slots = 0, vcap = 0, bcap = 0;
    int K = 0, nf = 1, e_words = 1, E_cap = 0;

    SceneDev S{};
    Tree st, dy, rxt, ets, etd;
    TriP *st_prims = nullptr, *dy_prims = nullptr;
    QNode4* st4 = nullptr;     // [T] the static tree as 4-wide quantised nodes
    int st4_n = 0;
    float4 *rx_prims = nullptr, *edge_prims = nullptr;
    float *box_st = nullptr, *box_dy = nullptr, *box_rx = nullptr, *box_ed = nullptr;
    BuildTemp tmp{};
    RaySoA rays[2]{};
    // regrouping between bounces: keys of the appended rays, the counting
    // sort's temp, which buffer holds bounce k's input (k + ray_flip) & 1, and
    // the key grid over the scene's x, y extent
    uint16_t* ray_key = nullptr;
    uint32_t* rg_temp = nullptr;
    int ray_flip = 0;
    bool regroup_now = false;
    float key_ox = 0.0f, key_oy = 0.0f, key_sx = 0.0f, key_sy = 0.0f;
    int* hitlog = nullptr;
    uint8_t* depth = nullptr;  // [n_total] bounce at which each ray of the last discovery launch ended
    unsigned long long* fresh = nullptr;  // [P] transmitter-side diffraction keys, in the order made
    // last step's end points and static line-of-sight tests (reused when nothing moved)
    double *prev_tx = nullptr, *prev_rx = nullptr;
    uint8_t *moved_tx = nullptr, *moved_rx = nullptr, *los_sb = nullptr;
    uint32_t* hist = nullptr;  // device flag: 1 once a step has run on this scene and cache
    uint32_t* dir_perm = nullptr;  // launch slot -> direction index (direction-Morton order)
    uint32_t* dir_slot = nullptr;  // direction index -> launch slot
    float4* dirs = nullptr;        // [rays_per_tx] launch directions in launch order
    unsigned long long* ctr = nullptr;
    unsigned long long* table = nullptr;
    KeyRec* cand = nullptr;
    KeyRec* cache[2] = {nullptr, nullptr};
    int cur = 0;
    uint32_t* illum = nullptr;
    ValidPaths vp{};
    LegBuf legs{};
    uint8_t* kstate = nullptr;
    uint32_t* occl = nullptr;
    uint32_t *sv0 = nullptr, *sv1 = nullptr;  // valid paths grouped by link, then in key order per link
    uint32_t* order = nullptr;
    int *link_start = nullptr, *link_end = nullptr;
    uint32_t *link_cnt = nullptr, *link_off = nullptr, *scan_tmp = nullptr;
    double* chan = nullptr;
    double *f_tx = nullptr, *f_txv = nullptr, *f_txo = nullptr, *f_rx = nullptr, *f_rxv = nullptr, *f_xf = nullptr,
           *f_ov = nullptr;
    // emrt_set_frame_host: device staging [8 n_tx + 6 n_rx + 15 n_objects], the
    // pinned host buffer it is uploaded from, and the event of the last upload
    double* f_stage = nullptr;
    double* fr_pin = nullptr;
    size_t fr_pin_n = 0;
    hipEvent_t ev_fr = nullptr;
    bool fr_pending = false;
    double* mat = nullptr;
    std::vector<double> mat_host;
    double* refl = nullptr;          // [kMaxMaterials] constant reflection magnitudes (0: Fresnel)
    std::vector<double> refl_host;
    uint32_t* flags = nullptr;
    uint32_t* scene_scratch = nullptr;
    int *obj_off = nullptr, *obj_faces = nullptr;
    uint8_t* obj_dyn = nullptr;
    uint32_t flag_accum = 0;
    int64_t frame_idx = -1;
    hipError_t pending = hipSuccess;  // first error of an unchecked async call
    // receiver-side launch: transmitter spheres and the launch's receivers
    Tree txt;
    float4* tx_prims = nullptr;
    float* box_tx = nullptr;
    int* rev_rx = nullptr;           // [kMaxRxSources]
    double* rev_pos = nullptr;       // [kMaxRxSources][3]
    std::vector<int> rev_host;
    int rev_n = 0, rev_rays = 0;     // nonzero only while a receiver-side step is enqueued
    bool last_rev = false;           // the hit log holds a receiver-side launch
    // reflection-diffraction candidates (diffraction = 2)
    unsigned long long* pairs = nullptr;  // [pair_slots] set of lit (source, face, edge)
    unsigned long long* pair_list = nullptr;
    long long pair_slots = 0;
    KeyRec* extra = nullptr;              // [P] proposed keys, referenced from the path table
    double st_area = 0.0;            // static tree quality (emrt_stats.static_tree_area)
};

#define HC(expr)                                                         \
    do {                                                                 \
        hipError_t e_ = (expr);                                          \
        if (e_ != hipSuccess && c->pending == hipSuccess) c->pending = e_; \
    } while (0)

static int32_t fail(emrt_ctx* c, int32_t code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

static int32_t hip_check(emrt_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess && c && c->pending != hipSuccess) {
        e = c->pending;
        c->pending = hipSuccess;
    }
    if (e == hipSuccess) return EMRT_OK;
    return fail(c, EMRT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------ layout ----
static void layout(emrt_ctx* c, Carver& cv) {
    const emrt_sizes& z = c->sz;
    long long V = z.n_verts, T = z.n_tris, F = z.n_faces, O = z.n_objects;
    SceneDev& S = c->S;
    S.verts_local_copy = cv.take<float>(3 * V);
    S.verts = cv.take<float>(3 * V);
    S.tris = cv.take<int>(3 * T);
    S.tri_face = cv.take<int>(T);
    S.face_object = cv.take<int>(F);
    S.face_material = cv.take<int>(F);
    S.face_dyn = cv.take<int>(F);
    S.vert_dyn = cv.take<int>(V);
    S.obj_rank = cv.take<int>(O);
    S.plane = cv.take<double>(4 * F);
    S.face_first = cv.take<int>(F);
    S.face_off = cv.take<int>(F + 1);
    S.face_tris = cv.take<int>(T);
    S.face_tv = cv.take<float>(9 * T);
    S.face_box = cv.take<float>(6 * F);
    S.tris_static = cv.take<int>(T);
    S.tris_dynamic = cv.take<int>(T);
    S.edge_i = cv.take<int>(2 * 6 * (long long)c->E_cap);
    S.edge_n = cv.take<double>(2 * (long long)c->E_cap);
    S.edges_static = cv.take<int>(c->E_cap);
    S.edges_dynamic = cv.take<int>(c->E_cap);
    c->obj_dyn = cv.take<uint8_t>(O);
    c->obj_off = cv.take<int>(O + 1);
    c->obj_faces = cv.take<int>(F);
    long long big = std::max(std::max(std::max(T, O), F), (long long)c->E_cap);
    c->scene_scratch = cv.take<uint32_t>(3 * big + 16 + (long long)scan_temp_bytes(big) / 4 + 64);
    // trees: worst case every triangle in one tree
    auto tree = [&](Tree& t, long long n) {
        long long ni = n > 1 ? n - 1 : 1;
        t.nodes = cv.take<BNode>(ni);
        t.leaf_parent = cv.take<int>(n);
        t.counters = cv.take<uint32_t>(ni);
        t.perm = cv.take<uint32_t>(n);
        t.span = cv.take<int>(ni);
        t.cap = (int)n;
    };
    tree(c->st, T);
    tree(c->dy, T);
    tree(c->rxt, z.n_rx);
    tree(c->ets, c->E_cap);
    tree(c->etd, c->E_cap);
    tree(c->txt, z.n_tx);
    c->st4 = cv.take<QNode4>(T);
    c->st_prims = cv.take<TriP>(T);
    c->dy_prims = cv.take<TriP>(T);
    c->rx_prims = cv.take<float4>(z.n_rx);
    c->edge_prims = cv.take<float4>(2LL * c->E_cap);
    c->box_st = cv.take<float>(6 * T);
    c->box_dy = cv.take<float>(6 * T);
    c->box_rx = cv.take<float>(6LL * z.n_rx);
    c->box_ed = cv.take<float>(6LL * c->E_cap);
    c->tx_prims = cv.take<float4>(z.n_tx);
    c->box_tx = cv.take<float>(6LL * z.n_tx);
    c->rev_rx = cv.take<int>(kMaxRxSources);
    c->rev_pos = cv.take<double>(3LL * kMaxRxSources);
    char* bt = cv.take<char>((long long)build_temp_bytes(c->bcap));
    if (!cv.measure) carve_build_temp(bt, c->bcap, c->tmp);
    for (int k = 0; k < 2; k++) {
        RaySoA& r = c->rays[k];
        r.ox = cv.take<float>(c->n_total); r.oy = cv.take<float>(c->n_total); r.oz = cv.take<float>(c->n_total);
        r.dx = cv.take<float>(c->n_total); r.dy = cv.take<float>(c->n_total); r.dz = cv.take<float>(c->n_total);
        r.L = cv.take<float>(c->n_total);
        r.id = cv.take<uint32_t>(c->n_total);
        r.prev = cv.take<int>(c->n_total);
    }
    if (c->cfg.ray_regroup && c->K >= 2) {
        c->ray_key = cv.take<uint16_t>(c->n_total);
        c->rg_temp = cv.take<uint32_t>((long long)regroup_temp_u32(c->n_total));
    }
    c->dyq_dev = cv.take<double>(2);
    c->hitlog = cv.take<int>((long long)(c->K + 1) * c->n_total);
    c->depth = cv.take<uint8_t>(c->n_total);
    c->dbg_sel = cv.take<uint32_t>(c->n_total / 32 + 1);
    c->dbg_log = cv.take<int>(3LL * EMRT_CAPTURE_LOG_ROWS);
    c->dbg_n = cv.take<unsigned long long>(1);
    c->dir_perm = cv.take<uint32_t>(c->cfg.rays_per_tx);
    c->dir_slot = cv.take<uint32_t>(c->cfg.rays_per_tx);
    c->dirs = cv.take<float4>(c->cfg.rays_per_tx);
    c->ctr = cv.take<unsigned long long>(kNumCounters);
    c->table = cv.take<unsigned long long>(c->table_slots);
    c->fresh = cv.take<unsigned long long>(c->P);
    c->prev_tx = cv.take<double>(3LL * z.n_tx);
    c->prev_rx = cv.take<double>(3LL * z.n_rx);
    c->moved_tx = cv.take<uint8_t>(z.n_tx);
    c->moved_rx = cv.take<uint8_t>(z.n_rx);
    c->los_sb = cv.take<uint8_t>(c->n_links);
    c->hist = cv.take<uint32_t>(1);
    const long long cw = compact_temp_elems((unsigned long long)c->table_slots);
    c->ctmp.flags = cv.take<uint32_t>(cw);
    c->ctmp.off = cv.take<uint32_t>(cw);
    c->ctmp.scan_tmp = cv.take<uint32_t>((long long)scan_temp_bytes(cw) / 4 + 16);
    c->cand = cv.take<KeyRec>(c->P);
    c->cache[0] = cv.take<KeyRec>(c->P);
    c->cache[1] = cv.take<KeyRec>(c->P);
    c->illum = cv.take<uint32_t>((long long)std::max<long long>(z.n_tx, kMaxRxSources) * c->e_words);
    if (c->pair_slots > 0) {
        c->pairs = cv.take<unsigned long long>(c->pair_slots);
        c->pair_list = cv.take<unsigned long long>(c->pair_slots);
        c->extra = cv.take<KeyRec>(c->P);
    }
    {
        const long long nc = (long long)kGridN * kGridN;
        c->bins.grid = cv.take<RxGrid>(1);
        c->bins.cnt = cv.take<uint32_t>(nc);
        c->bins.cursor = cv.take<uint32_t>(nc);
        c->bins.start = cv.take<uint32_t>(nc + 1);
        c->bins.scan_tmp = cv.take<uint32_t>((long long)scan_temp_bytes(nc) / 4 + 16);
        c->bins.sorted = cv.take<float4>(z.n_rx);
    }
    ValidPaths& vp = c->vp;
    vp.cap = c->vcap;
    vp.key = cv.take<KeyRec>(c->vcap);
    vp.tri = cv.take<int>(5 * c->vcap);
    vp.a = cv.take<double>(2LL * c->nf * c->vcap);
    vp.tau = cv.take<double>(c->vcap);
    vp.fd = cv.take<double>((long long)c->nf * c->vcap);
    vp.ang = cv.take<float4>(c->vcap);
    c->sv0 = cv.take<uint32_t>(c->vcap);
    c->sv1 = cv.take<uint32_t>(c->vcap);
    LegBuf& lg = c->legs;
    lg.cap = 3 * c->vcap;
    lg.cap_first = c->vcap;  // one receiver leg per key slot
    // the shadow legs live only during a step's validation; emrt_backward
    // reuses their block for its per-path partial derivatives (15 doubles per
    // path slot: the same 120 bytes as three legs)
    {
        const long long n = lg.cap;
        char* blk = cv.take<char>(40LL * n + 10LL * 256);
        c->leg_block = blk;
        if (!cv.measure) {
            auto carve = [&](long long k) { return (void*)(blk + k * (((4LL * n) + 255) / 256 * 256)); };
            lg.ox = (float*)carve(0); lg.oy = (float*)carve(1); lg.oz = (float*)carve(2);
            lg.dx = (float*)carve(3); lg.dy = (float*)carve(4); lg.dz = (float*)carve(5);
            lg.xa = (int*)carve(6);
            lg.xb = (int*)carve(7);
            lg.xc = (int*)carve(8);
            lg.key = (uint32_t*)carve(9);
        }
    }
    lg.list = cv.take<uint32_t>(lg.cap - lg.cap_first);
    c->kstate = cv.take<uint8_t>(c->vcap);
    c->occl = cv.take<uint32_t>(c->vcap);
    c->vtmp.flag = cv.take<uint32_t>(c->vcap);
    c->vtmp.off = cv.take<uint32_t>(c->vcap);
    c->vtmp.flag_d = cv.take<uint32_t>(c->vcap);
    c->vtmp.off_d = cv.take<uint32_t>(c->vcap);
    c->vtmp.flag_r = cv.take<uint32_t>(c->vcap);
    c->vtmp.off_r = cv.take<uint32_t>(c->vcap);
    c->vtmp.cnt = cv.take<uint32_t>(3);
    c->vtmp.surv = cv.take<uint32_t>(c->vcap);
    c->ktri = cv.take<int>(5 * c->vcap);
    c->vtmp.scan_tmp = cv.take<uint32_t>((long long)scan_temp_bytes(c->vcap) / 4 + 16);
    c->link_start = cv.take<int>(c->n_links);
    c->link_end = cv.take<int>(c->n_links);
    c->link_cnt = cv.take<uint32_t>(c->n_links);
    c->link_off = cv.take<uint32_t>(c->n_links);
    c->scan_tmp = cv.take<uint32_t>((long long)scan_temp_bytes(c->n_links) / 4 + 16);
    c->chan = cv.take<double>(8LL * c->nf * c->n_links + c->n_links + 8);
    c->f_tx = cv.take<double>(3LL * z.n_tx);
    c->f_txv = cv.take<double>(3LL * z.n_tx);
    c->f_txo = cv.take<double>(2LL * z.n_tx);
    c->f_rx = cv.take<double>(3LL * z.n_rx);
    c->f_rxv = cv.take<double>(3LL * z.n_rx);
    c->f_xf = cv.take<double>(12 * O);
    c->f_ov = cv.take<double>(3 * O);
    c->f_stage = cv.take<double>(8LL * z.n_tx + 6LL * z.n_rx + 15 * O);
    c->mat = cv.take<double>(2 * kMaxMaterials);
    c->refl = cv.take<double>(kMaxMaterials);
    c->flags = cv.take<uint32_t>(16);
    {
        long long nl = c->n_links, nfl = (long long)c->nf * nl;
        c->coh.frames = cv.take<unsigned long long>(1);
        c->coh.ring = cv.take<double>(nfl * EMRT_CORR_LAGS);
        c->coh.prod = cv.take<double>(nfl * EMRT_CORR_LAGS);
        c->coh.s1 = cv.take<double>(nfl);
        c->coh.s2 = cv.take<double>(nfl);
        c->coh.prev_los = cv.take<uint32_t>(nl);
        c->coh.prev_hash = cv.take<unsigned long long>(nl);
        c->coh.trigger = cv.take<uint32_t>(nl);
    }
    if (c->cfg.adjoint_materials > 0) c->adj_rows = cv.take<double>((5LL + 2LL * c->cfg.adjoint_materials) * c->n_links);
    if (!cv.measure) c->vp.count = c->ctr + C_NVALID;
}

static void derive(emrt_ctx* c) {
    const emrt_sizes& z = c->sz;
    c->K = c->cfg.max_reflections;
    c->nf = c->cfg.n_freq;
    c->n_total = (long long)z.n_tx * c->cfg.rays_per_tx;
    c->n_links = (long long)z.n_tx * z.n_rx;
    c->P = c->cfg.path_capacity;
    c->table_slots = pow2_at_least(std::max<int64_t>(c->cfg.table_capacity, 1024));
    c->vcap = c->n_links + c->P;
    c->E_cap = (int)std::min<long long>(3LL * z.n_faces + 16, (1LL << 24) - 1);
    c->e_words = (c->E_cap + 31) / 32;
    long long b = std::max<long long>({z.n_tris, (long long)c->E_cap, (long long)z.n_rx, (long long)z.n_tx,
                                       (long long)c->cfg.rays_per_tx, z.n_faces, z.n_objects, 16LL});
    b = std::max<long long>(b, z.n_tris + c->E_cap + std::max<long long>(z.n_rx, z.n_tx));  // one batched build
    c->bcap = b;
    c->pair_slots = c->cfg.diffraction == 2 ? pow2_at_least(std::max<int64_t>(c->cfg.table_capacity / 4, 1 << 16)) : 0;
}

static void coherence_clear(emrt_ctx* c);

// ---------------------------------------------------------------- ABI ----
extern "C" {

void emrt_config_default(emrt_config* cfg) {
    if (!cfg) return;
    memset(cfg, 0, sizeof(*cfg));
    cfg->n_freq = 1;
    cfg->freq_hz[0] = 28e9;
    cfg->max_reflections = 3;
    cfg->diffraction = 0;
    cfg->rays_per_tx = 10000;
    cfg->rx_sphere_k = 1.0;
    cfg->diff_max_leg_m = 250.0;
    cfg->tx_power_w = 100.0;
    cfg->antenna_mode = EMRT_ANT_ISO_V;
    cfg->path_cap_per_link = 64;
    cfg->path_capacity = 4LL << 20;
    cfg->table_capacity = 0;
    cfg->ray_regroup = 0;
    cfg->dyn_rebuild_ratio = 0.0;
}

int32_t emrt_ctx_create(const emrt_config* cfg, emrt_ctx** out) {
    if (!cfg || !out) return EMRT_E_INVALID;
    *out = nullptr;
    if (cfg->n_freq < 1 || cfg->n_freq > 4 || cfg->max_reflections < 0 || cfg->max_reflections > 5)
        return EMRT_E_UNSUPPORTED;
    if (cfg->rays_per_tx < 1 || !(cfg->rx_sphere_k > 0) || !(cfg->diff_max_leg_m >= 0) || cfg->path_capacity < 1 ||
        cfg->path_capacity > (1LL << 31) || cfg->antenna_mode < 0 || cfg->antenna_mode > 1 ||
        cfg->adjoint_materials < 0 || cfg->adjoint_materials > kMaxMaterials || cfg->diffraction < 0 ||
        cfg->diffraction > 2 || (cfg->ray_regroup != 0 && cfg->ray_regroup != 1) || !(cfg->dyn_rebuild_ratio >= 0.0))
        return EMRT_E_INVALID;
    // one reflection combined with one diffraction: the kernels below are
    // complete (k_pair_list, k_pair_cand, the combined construction and
    // fields) but the configuration stays refused until they have run clean
    if (cfg->diffraction == 2) return EMRT_E_UNSUPPORTED;
    for (int i = 0; i < cfg->n_freq; i++)
        if (!(cfg->freq_hz[i] > 0)) return EMRT_E_INVALID;
    emrt_ctx* c = new emrt_ctx();
    c->cfg = *cfg;
    if (c->cfg.table_capacity <= 0) c->cfg.table_capacity = 4 * c->cfg.path_capacity;
    if (c->cfg.path_cap_per_link <= 0) c->cfg.path_cap_per_link = 64;
    *out = c;
    return EMRT_OK;
}

int32_t emrt_ctx_destroy(emrt_ctx* c) {
    if (!c) return EMRT_E_INVALID;
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->ev_dyq) (void)hipEventDestroy(c->ev_dyq);
    if (c->ev_fr) (void)hipEventDestroy(c->ev_fr);
    if (c->fr_pin) (void)hipHostFree(c->fr_pin);
    if (c->dyq_host) (void)hipHostFree(c->dyq_host);
    if (c->ev_created)
        for (auto& set : c->evs)
            for (auto e : set.ev) (void)hipEventDestroy(e);
    delete c;
    return EMRT_OK;
}

int32_t emrt_workspace_size(emrt_ctx* c, const emrt_sizes* s, size_t* bytes) {
    if (!c || !s || !bytes) return fail(c, EMRT_E_INVALID, "null argument");
    if (s->n_verts < 3 || s->n_tris < 1 || s->n_faces < 1 || s->n_objects < 1 || s->n_tx < 1 || s->n_rx < 1)
        return fail(c, EMRT_E_INVALID, "sizes must be positive");
    if (s->n_tris >= (1LL << 31) || s->n_verts >= (1LL << 31) || s->n_tx > 4095 || s->n_rx >= (1 << 26))
        return fail(c, EMRT_E_UNSUPPORTED, "scene too large (n_tx <= 4095, n_rx < 2^26, n_tris < 2^31)");
    if ((long long)s->n_tx * c->cfg.rays_per_tx >= (1LL << 32))
        return fail(c, EMRT_E_UNSUPPORTED, "n_tx * rays_per_tx must be below 2^32");
    if ((long long)s->n_tx * s->n_rx + c->cfg.path_capacity >= (1LL << 31))  // key slots are 31-bit
        return fail(c, EMRT_E_UNSUPPORTED, "n_tx * n_rx + path_capacity must be below 2^31");
    c->sz = *s;
    c->sized = true;
    derive(c);
    Carver cv(nullptr);
    layout(c, cv);
    *bytes = cv.off + 256;
    return EMRT_OK;
}

int32_t emrt_bind_workspace(emrt_ctx* c, void* ptr, size_t bytes) {
    if (!c) return EMRT_E_INVALID;
    if (!c->sized) return fail(c, EMRT_E_STATE, "call emrt_workspace_size first");
    if (!ptr) return fail(c, EMRT_E_WORKSPACE, "null workspace");
    Carver m(nullptr);
    layout(c, m);
    char* base = (char*)(((uintptr_t)ptr + 255) & ~(uintptr_t)255);
    size_t need = m.off + (size_t)(base - (char*)ptr);
    if (bytes < need) return fail(c, EMRT_E_WORKSPACE, "workspace too small");
    Carver cv(base);
    layout(c, cv);
    c->ws = (char*)ptr;
    c->ws_bytes = bytes;
    c->bound = true;
    c->scene_set = c->frame_set = c->stepped = false;
    fill_u64(c->ctr, 0ULL, kNumCounters, c->stream);
    fill_u32(c->flags, 0u, 16, c->stream);
    fill_u32(c->hist, 0u, 1, c->stream);
    fill_u32(c->dbg_sel, 0u, c->n_total / 32 + 1, c->stream);
    fill_u64(c->dbg_n, 0ULL, 1, c->stream);
    c->dbg_on = false;
    coherence_clear(c);
    return EMRT_OK;
}

// ---------------------------------------------- static workspace ----
// A workspace held by the library itself, for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).  Each GPU the library runs on holds its own copy of the
// array until the process ends.  Its device address comes from
// hipGetSymbolAddress, once per device, on the first bind on that device; the
// array's name is a host-side stand-in and is never passed to a kernel or a
// copy.  Every context bound to it on one GPU shares the same memory, so only
// one such context per GPU may be in use at a time (a later bind takes it
// over; overlapping use races).  The bind clears the counters and flags that
// must start at zero, as emrt_bind_workspace does for any workspace.
static __device__ __align__(256) unsigned char scratch[EMRT_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

int32_t emrt_bind_static_workspace(emrt_ctx* c) {
    if (!c) return EMRT_E_INVALID;
    if (!c->sized) return fail(c, EMRT_E_STATE, "call emrt_workspace_size first");
    Carver m(nullptr);
    layout(c, m);
    const size_t need = m.off + 256;
    if (need > (size_t)EMRT_STATIC_WORKSPACE_BYTES)
        return fail(c, EMRT_E_WORKSPACE, "the sizes need a workspace of " + std::to_string(need) +
                                             " bytes; the static workspace holds " +
                                             std::to_string((size_t)EMRT_STATIC_WORKSPACE_BYTES) +
                                             " (use emrt_bind_workspace with a caller buffer)");
    void* p = nullptr;
    hipError_t e = scratch_address(&p);
    if (e != hipSuccess) return fail(c, EMRT_E_HIP, std::string("static workspace address: ") + hipGetErrorString(e));
    return emrt_bind_workspace(c, p, (size_t)EMRT_STATIC_WORKSPACE_BYTES);
}

int32_t emrt_set_stream(emrt_ctx* c, void* s) {
    if (!c) return EMRT_E_INVALID;
    c->stream = (hipStream_t)s;
    return EMRT_OK;
}

int32_t emrt_set_materials(emrt_ctx* c, const double* eps, int32_t M) {
    if (!c || !eps || M < 1 || M > kMaxMaterials) return fail(c, EMRT_E_INVALID, "bad material table");
    if (!c->bound) return fail(c, EMRT_E_STATE, "no workspace");
    for (int i = 0; i < 2 * M; i++)
        if (!std::isfinite(eps[i])) return fail(c, EMRT_E_INVALID, "non-finite permittivity");
    c->mat_host.assign(eps, eps + 2 * M);
    c->S.M = M;
    return hip_check(c, hipMemcpyAsync(c->mat, c->mat_host.data(), sizeof(double) * 2 * M, hipMemcpyHostToDevice,
                                       c->stream), "material upload");
}

int32_t emrt_set_reflection_coefficients(emrt_ctx* c, const double* refl, int32_t M) {
    if (!c || !refl) return fail(c, EMRT_E_INVALID, "null reflection table");
    if (!c->bound || c->S.M < 1) return fail(c, EMRT_E_STATE, "no scene");
    if (M != c->S.M) return fail(c, EMRT_E_INVALID, "reflection table size differs from the material count");
    for (int i = 0; i < M; i++)
        if (!(refl[i] >= 0.0 && refl[i] <= 1.0)) return fail(c, EMRT_E_INVALID, "reflection coefficient outside [0, 1]");
    c->refl_host.assign(kMaxMaterials, 0.0);
    std::copy(refl, refl + M, c->refl_host.begin());
    return hip_check(c, hipMemcpyAsync(c->refl, c->refl_host.data(), sizeof(double) * kMaxMaterials,
                                       hipMemcpyHostToDevice, c->stream),
                     "reflection table upload");
}

static void coherence_clear(emrt_ctx* c) {
    long long nl = c->n_links, nfl = (long long)c->nf * nl;
    hipStream_t st = c->stream;
    fill_u64(c->coh.frames, 0ULL, 1, st);
    fill_u64((unsigned long long*)c->coh.ring, 0ULL, nfl * EMRT_CORR_LAGS, st);
    fill_u64((unsigned long long*)c->coh.prod, 0ULL, nfl * EMRT_CORR_LAGS, st);
    fill_u64((unsigned long long*)c->coh.s1, 0ULL, nfl, st);
    fill_u64((unsigned long long*)c->coh.s2, 0ULL, nfl, st);
    fill_u32(c->coh.prev_los, 0u, nl, st);
    fill_u64(c->coh.prev_hash, 0ULL, nl, st);
    fill_u32(c->coh.trigger, 0u, nl, st);
}

static int32_t sync_read(emrt_ctx* c, void* dst, const void* src, size_t n) {
    hipError_t e = hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_check(c, e, "device read");
}

int32_t emrt_set_scene(emrt_ctx* c, const emrt_scene_desc* d) {
    if (!c || !d) return EMRT_E_INVALID;
    if (!c->bound) return fail(c, EMRT_E_STATE, "no workspace bound");
    const emrt_sizes& z = c->sz;
    if (d->n_verts != z.n_verts || d->n_tris != z.n_tris || d->n_faces != z.n_faces || d->n_objects != z.n_objects)
        return fail(c, EMRT_E_INVALID, "scene sizes differ from the workspace sizes");
    if (!d->verts || !d->tris || !d->tri_face || !d->face_object || !d->face_material || !d->object_dynamic)
        return fail(c, EMRT_E_INVALID, "null scene array");
    int32_t rc = emrt_set_materials(c, d->material_eps, d->n_materials);
    if (rc) return rc;
    c->refl_host.assign(kMaxMaterials, 0.0);
    HC(hipMemcpyAsync(c->refl, c->refl_host.data(), sizeof(double) * kMaxMaterials, hipMemcpyHostToDevice,
                      c->stream));
    hipStream_t st = c->stream;
    SceneDev& S = c->S;
    S.V = (int)z.n_verts; S.T = (int)z.n_tris; S.F = (int)z.n_faces; S.O = (int)z.n_objects;
    S.E_cap = c->E_cap;
    HC(hipMemcpyAsync(S.verts_local_copy, d->verts, sizeof(float) * 3 * z.n_verts, hipMemcpyDeviceToDevice, st));
    HC(hipMemcpyAsync(S.verts, d->verts, sizeof(float) * 3 * z.n_verts, hipMemcpyDeviceToDevice, st));
    HC(hipMemcpyAsync(S.tris, d->tris, sizeof(int) * 3 * z.n_tris, hipMemcpyDeviceToDevice, st));
    HC(hipMemcpyAsync(S.tri_face, d->tri_face, sizeof(int) * z.n_tris, hipMemcpyDeviceToDevice, st));
    HC(hipMemcpyAsync(S.face_object, d->face_object, sizeof(int) * z.n_faces, hipMemcpyDeviceToDevice, st));
    HC(hipMemcpyAsync(S.face_material, d->face_material, sizeof(int) * z.n_faces, hipMemcpyDeviceToDevice, st));
    HC(hipMemcpyAsync(c->obj_dyn, d->object_dynamic, z.n_objects, hipMemcpyDeviceToDevice, st));
    fill_u32(c->flags, 0u, 16, st);
    scene_check(S, c->obj_dyn, c->flags, st);
    uint32_t fl = 0;
    if ((rc = sync_read(c, &fl, c->flags, sizeof(fl)))) return rc;
    if (fl & FLAG_BAD_INPUT)
        return fail(c, EMRT_E_INVALID, "scene: index out of range, degenerate or non-finite triangle");
    int* counts = (int*)(c->ctr + C_SCRATCH);
    scene_prepare(S, c->obj_dyn, c->scene_scratch, counts, c->tmp, st);
    int cnt[2] = {0, 0};
    if ((rc = sync_read(c, cnt, counts, sizeof(cnt)))) return rc;
    S.O_d = cnt[0];
    S.T_s = cnt[1];
    S.T_d = S.T - S.T_s;
    int E = scene_edges(S, c->obj_off, c->obj_faces, counts + 4, c->tmp, st);
    if (E < 0) return fail(c, EMRT_E_UNSUPPORTED, "too many wedge edges");
    // edges of static objects in a tree built once (below), those of moving ones per frame
    if (edge_partition(S, c->scene_scratch, counts + 6, st) < 0) return fail(c, EMRT_E_HIP, "edge partition");
    // static tree (world == local for static vertices)
    scene_planes(S, st);
    tri_boxes(S, S.tris_static, S.T_s, c->box_st, st);
    if (bvh_build_sah(c->box_st, S.T_s, c->st, c->tmp, st) < 0) return fail(c, EMRT_E_HIP, "static tree build");
    tri_prims(S, S.tris_static, c->st, c->st_prims, st);
    c->st4_n = 0;
    if (S.T_s > 0) {  // the same tree as 4-wide quantised nodes (collapsed on the host, once per scene)
        const int nb = std::max(S.T_s - 1, 1);
        std::vector<BNode> hb((size_t)nb);
        std::vector<QNode4> h4((size_t)nb);
        if ((rc = sync_read(c, hb.data(), c->st.nodes, sizeof(BNode) * (size_t)nb))) return rc;
        const int n4 = bvh4_collapse(hb.data(), S.T_s, h4.data(), nb);
        if (n4 < 1) return fail(c, EMRT_E_HIP, "static tree collapse");
        HC(hipMemcpyAsync(c->st4, h4.data(), sizeof(QNode4) * (size_t)n4, hipMemcpyHostToDevice, st));
        HC(hipStreamSynchronize(st));  // h4 is a host temporary
        c->st4_n = n4;
    }
    // regroup key grid: the static scene's x, y extent in 16 cells per axis
    c->key_ox = c->key_oy = c->key_sx = c->key_sy = 0.0f;
    if (S.T_s >= 2) {
        BNode root;
        if ((rc = sync_read(c, &root, c->st.nodes, sizeof(root)))) return rc;
        const float lx = fminf(root.a.x, root.b.z), ly = fminf(root.a.y, root.b.w);
        const float hx = fmaxf(root.a.w, root.c.y), hy = fmaxf(root.b.x, root.c.z);
        c->key_ox = lx;
        c->key_oy = ly;
        c->key_sx = hx > lx ? 16.0f / (hx - lx) : 0.0f;
        c->key_sy = hy > ly ? 16.0f / (hy - ly) : 0.0f;
    }
    // static edges: binned SAH once per scene (the tree the reception cones of
    // every primary ray walk), their primitives at the front of edge_prims
    c->ets.n = 0;
    if (S.E_s > 0) {
        edge_boxes(S, S.edges_static, S.E_s, c->box_ed, st);
        if (bvh_build_sah(c->box_ed, S.E_s, c->ets, c->tmp, st) < 0) return fail(c, EMRT_E_HIP, "static edge tree build");
        edge_prims(S, S.edges_static, c->ets, c->edge_prims, st);
    }
    c->st_area = 0.0;
    if (S.T_s > 1) {  // tree quality: child box areas over the root box area
        double* acc = (double*)c->tmp.bounds;
        fill_u64((unsigned long long*)acc, 0ULL, 1, st);
        bvh_sah(c->st, acc, st);
        double sum = 0.0;
        BNode root;
        if ((rc = sync_read(c, &sum, acc, sizeof(sum)))) return rc;
        if ((rc = sync_read(c, &root, c->st.nodes, sizeof(root)))) return rc;
        double lo[3] = {std::min(root.a.x, root.b.z), std::min(root.a.y, root.b.w), std::min(root.a.z, root.c.x)};
        double hi[3] = {std::max(root.a.w, root.c.y), std::max(root.b.x, root.c.z), std::max(root.b.y, root.c.w)};
        double ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
        double ra = 2.0 * (ex * ey + ey * ez + ez * ex);
        c->st_area = ra > 0.0 ? sum / ra : 0.0;
    }
    c->dy.n = 0;  // the first frame builds the moving objects' tree
    c->dyq_pending = false;
    c->dyq_built = c->dyq_last = 0.0;
    c->dyn_rebuilds = 0;
    ray_order(c->cfg.rays_per_tx, c->dir_perm, c->tmp, st);
    invert_perm(c->dir_perm, c->dir_slot, c->cfg.rays_per_tx, st);
    dir_table(c->dir_perm, c->cfg.rays_per_tx, c->dirs, st);
    // empty cache
    fill_u32(c->hist, 0u, 1, st);  // a new scene: nothing from an earlier step carries over
    fill_u64(c->ctr, 0ULL, kNumCounters, st);
    c->cur = 0;
    c->scene_set = true;
    c->frame_set = c->stepped = c->discovered = false;
    c->frame_idx = -1;
    return hip_check(c, hipStreamSynchronize(st), "set_scene");
}

// The frame's arrays into the context in one launch (up to seven device
// arrays of doubles; a null source writes zeros).
struct FrameCopy {
    const double* src[7];
    double* dst[7];
    long long n[7];
    int k;
};

__global__ void k_frame_copy(FrameCopy fc) {
    long long total = 0;
    for (int j = 0; j < fc.k; j++) total += fc.n[j];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        long long r = i;
        int j = 0;
        while (r >= fc.n[j]) r -= fc.n[j++];
        fc.dst[j][r] = fc.src[j] ? fc.src[j][r] : 0.0;
    }
}

static int32_t frame_check(emrt_ctx* c, const emrt_frame_desc* f) {
    if (!c || !f) return EMRT_E_INVALID;
    if (!c->scene_set) return fail(c, EMRT_E_STATE, "set_scene first");
    if (f->n_tx != c->sz.n_tx || f->n_rx != c->sz.n_rx) return fail(c, EMRT_E_INVALID, "n_tx / n_rx differ from sizes");
    if (!f->tx_pos || !f->rx_pos || !f->tx_vel || !f->rx_vel) return fail(c, EMRT_E_INVALID, "null frame array");
    if (c->S.O_d > 0 && (!f->obj_xform || !f->obj_vel)) return fail(c, EMRT_E_INVALID, "dynamic objects need transforms");
    return EMRT_OK;
}

// the frame's device arrays into the context, in one launch
static int32_t frame_gather(emrt_ctx* c, const emrt_frame_desc* f) {
    hipStream_t st = c->stream;
    const long long ntx = c->sz.n_tx, nrx = c->sz.n_rx, nd = c->S.O_d;
    FrameCopy fc{};
    auto add = [&](const double* src, double* dst, long long n) {
        fc.src[fc.k] = src;
        fc.dst[fc.k] = dst;
        fc.n[fc.k++] = n;
    };
    add(f->tx_pos, c->f_tx, 3 * ntx);
    add(f->tx_vel, c->f_txv, 3 * ntx);
    add(f->tx_orient, c->f_txo, 2 * ntx);  // null: zeros
    add(f->rx_pos, c->f_rx, 3 * nrx);
    add(f->rx_vel, c->f_rxv, 3 * nrx);
    if (nd > 0) {
        add(f->obj_xform, c->f_xf, 12 * nd);
        add(f->obj_vel, c->f_ov, 3 * nd);
    }
    const long long total = 8 * ntx + 6 * nrx + 15 * nd;
    hipLaunchKernelGGL(k_frame_copy, dim3((unsigned)std::min<long long>((total + 255) / 256, 1024)), dim3(256), 0, st,
                       fc);
    c->frame_set = true;
    c->frame_since_step = true;
    c->frame_idx = f->frame;
    return hip_check(c, hipGetLastError(), "set_frame");
}

int32_t emrt_set_frame(emrt_ctx* c, const emrt_frame_desc* f) {
    int32_t rc = frame_check(c, f);
    if (rc) return rc;
    return frame_gather(c, f);
}

int32_t emrt_set_frame_host(emrt_ctx* c, const emrt_frame_desc* f) {
    int32_t rc = frame_check(c, f);
    if (rc) return rc;
    const long long ntx = c->sz.n_tx, nrx = c->sz.n_rx, nd = c->S.O_d;
    const size_t n = (size_t)(8 * ntx + 6 * nrx + 15 * nd);
    if (c->fr_pending) {  // the pinned buffer still feeds the previous upload
        HC(hipEventSynchronize(c->ev_fr));
        c->fr_pending = false;
    }
    if (!c->fr_pin || c->fr_pin_n < n) {
        if (c->fr_pin) (void)hipHostFree(c->fr_pin);
        c->fr_pin = nullptr;
        c->fr_pin_n = 0;
        if (hipHostMalloc((void**)&c->fr_pin, sizeof(double) * std::max<size_t>(n, 1), hipHostMallocDefault) != hipSuccess) {
            c->fr_pin = nullptr;
            return fail(c, EMRT_E_HIP, "pinned frame buffer");
        }
        c->fr_pin_n = n;
    }
    if (!c->ev_fr && hipEventCreateWithFlags(&c->ev_fr, hipEventDisableTiming) != hipSuccess) {
        c->ev_fr = nullptr;
        return fail(c, EMRT_E_HIP, "frame upload event");
    }
    // packed in the gather's order; a null orientation becomes zeros
    emrt_frame_desc d = *f;
    size_t off = 0;
    auto put = [&](const double* src, long long cnt) -> const double* {
        if (src) memcpy(c->fr_pin + off, src, sizeof(double) * (size_t)cnt);
        else memset(c->fr_pin + off, 0, sizeof(double) * (size_t)cnt);
        const double* dev = c->f_stage + off;
        off += (size_t)cnt;
        return dev;
    };
    d.tx_pos = put(f->tx_pos, 3 * ntx);
    d.tx_vel = put(f->tx_vel, 3 * ntx);
    d.tx_orient = put(f->tx_orient, 2 * ntx);
    d.rx_pos = put(f->rx_pos, 3 * nrx);
    d.rx_vel = put(f->rx_vel, 3 * nrx);
    if (nd > 0) {
        d.obj_xform = put(f->obj_xform, 12 * nd);
        d.obj_vel = put(f->obj_vel, 3 * nd);
    }
    HC(hipMemcpyAsync(c->f_stage, c->fr_pin, sizeof(double) * off, hipMemcpyHostToDevice, c->stream));
    const hipError_t er = hipEventRecord(c->ev_fr, c->stream);
    if (er != hipSuccess) {  // no event to wait on: the pinned buffer is free once the stream is
        (void)hipStreamSynchronize(c->stream);
        return hip_check(c, er, "frame upload event");
    }
    c->fr_pending = true;
    return frame_gather(c, &d);
}

static void ev_flush(emrt_ctx* c, emrt_ctx::EventSet& set) {
    if (!set.pending) return;
    set.pending = false;
    if (set.used == 0 || hipEventSynchronize(set.ev[set.used - 1]) != hipSuccess) return;
    for (int i = 0; i + 1 < set.bounce_end; i += 2) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, set.ev[i], set.ev[i + 1]) == hipSuccess) { c->t_bounce_ms += ms; c->t_bounce_n++; }
    }
    if (set.used - set.bounce_end >= 2) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, set.ev[set.bounce_end], set.ev[set.bounce_end + 1]) == hipSuccess) {
            c->t_validate_ms += ms;
            c->t_validate_n++;
        }
    }
}

static void ev_record(emrt_ctx* c) {
    if (!c->timing_on) return;
    auto& set = c->evs[c->ev_parity];
    if (set.used < 16) HC(hipEventRecord(set.ev[set.used++], c->stream));
}

int32_t emrt_set_instrumentation(emrt_ctx* c, int32_t stats, int32_t timing) {
    if (!c) return EMRT_E_INVALID;
    c->stats_on = stats ? 1 : 0;
    c->timing_on = timing ? 1 : 0;
    if (c->timing_on && !c->ev_created) {
        for (auto& set : c->evs)
            for (auto& e : set.ev)
                if (hipEventCreate(&e) != hipSuccess) return fail(c, EMRT_E_HIP, "event create");
        c->ev_created = true;
    }
    for (auto& set : c->evs) {
        ev_flush(c, set);
        set.used = set.bounce_end = 0;
    }
    c->t_bounce_ms = c->t_validate_ms = 0;
    c->t_bounce_n = c->t_validate_n = 0;
    return EMRT_OK;
}

static PathArgs path_args(emrt_ctx* c) {
    PathArgs a{};
    a.s = c->S;
    a.f.n_tx = c->sz.n_tx;
    a.f.n_rx = c->sz.n_rx;
    a.f.tx_pos = c->f_tx; a.f.tx_vel = c->f_txv; a.f.tx_orient = c->f_txo;
    a.f.rx_pos = c->f_rx; a.f.rx_vel = c->f_rxv; a.f.obj_vel = c->f_ov;
    a.st = c->st.view(); a.dy = c->dy.view();
    a.st4 = Bvh4{c->st4, c->S.T_s, c->st4_n};
    a.st_prims = c->st_prims; a.dy_prims = c->dy_prims;
    a.fc.mat_eps = c->mat;
    a.fc.mat_refl = c->refl;
    a.fc.nf = c->nf;
    for (int i = 0; i < EMRT_NF; i++) a.fc.freq[i] = i < c->nf ? c->cfg.freq_hz[i] : 1.0;
    a.fc.ant_mode = c->cfg.antenna_mode;
    a.diff_max_leg = c->cfg.diff_max_leg_m;
    a.combined = c->cfg.diffraction == 2 ? 1 : 0;
    a.out = c->vp;
    a.legs = c->legs;
    a.legs.count = c->ctr + C_NLEGS;
    a.legs.n_list = c->ctr + C_NLIST;
    a.state = c->kstate;
    a.occl = c->occl;
    a.moved_tx = c->moved_tx;
    a.moved_rx = c->moved_rx;
    a.los_sb = c->los_sb;
    a.ktri = c->ktri;
    a.flags = c->flags;
    return a;
}

// ---------------------------------------------------- step, in phases ----
// A step is enqueued in three phases so that batched stepping can run the
// bounces of several scenes in one launch: step_pre (frame geometry, trees,
// on discovery frames the table and the primary rays), the K + 1 bounces,
// and step_post (candidates, validation, fields, per-link sums, next cache).

// The discovery launch of the step being enqueued: from every transmitter,
// or (rev_n > 0) from the rev_n receivers of a receiver-side step.
static long long launch_total(const emrt_ctx* c) {
    return c->rev_n > 0 ? (long long)c->rev_n * c->rev_rays : c->n_total;
}
static FreshKeys fresh_keys(const emrt_ctx* c) { return FreshKeys{c->fresh, c->ctr + C_NFRESH, c->P}; }
static KeySrc key_src(const emrt_ctx* c, const KeyRec* cache) {
    const bool rev = c->rev_n > 0;
    return KeySrc{c->hitlog, c->S.tri_face, cache, launch_total(c), rev ? c->rev_rays : c->cfg.rays_per_tx,
                  rev ? c->rev_rx : nullptr, c->extra};
}

// Bounce arguments of level k; tree sizes are those the step's trees have
// once step_pre has run (so the arguments can be prepared in advance).
static BounceArgs bounce_args(emrt_ctx* c, int k, int parity) {
    SceneDev& S = c->S;
    bool diff = c->cfg.diffraction && S.E > 0;
    const bool rev = c->rev_n > 0;
    const int rays = rev ? c->rev_rays : c->cfg.rays_per_tx;
    BounceArgs b{};
    b.K = c->K;
    b.n_total = launch_total(c);
    if (c->regroup_now && c->ray_key && k >= 1 && k < c->K) {
        b.out_key = c->ray_key;
        b.key_ox = c->key_ox; b.key_oy = c->key_oy; b.key_sx = c->key_sx; b.key_sy = c->key_sy;
    }
    b.rays_per_tx = rays;
    b.st = Bvh{c->st.nodes, S.T_s};
    b.st4 = Bvh4{c->st4, S.T_s, c->st4_n};
    b.dy = Bvh{c->dy.nodes, S.T_d};
    b.st_prims = c->st_prims;
    b.dy_prims = c->dy_prims;
    b.plane = S.plane;
    b.rxt = rev ? Bvh{c->txt.nodes, c->sz.n_tx} : Bvh{c->rxt.nodes, c->sz.n_rx};
    b.rx_prims = rev ? c->tx_prims : c->rx_prims;
    b.alpha_k = (float)(c->cfg.rx_sphere_k * sqrt(4.0 * kPi / (double)rays));
    b.diffraction = diff ? c->cfg.diffraction : 0;
    b.pairs = c->pairs;
    b.pair_mask = c->pair_slots ? (unsigned long long)c->pair_slots - 1ULL : 0ULL;
    b.ets = Bvh{c->ets.nodes, diff ? S.E_s : 0};
    b.etd = Bvh{c->etd.nodes, diff ? S.E_dyn : 0};
    b.eprims_s = c->edge_prims;
    b.eprims_d = c->edge_prims + 2LL * S.E_s;
    b.illum = c->illum;
    b.e_words = c->e_words;
    b.table = c->table;
    b.mask = (unsigned long long)c->table_slots - 1ULL;
    b.src = key_src(c, c->cache[parity]);
    b.hitlog = c->hitlog;
    b.depth = c->depth;
    b.flags = c->flags;
    b.stats = c->ctr + C_STATS;
    b.b = k;
    b.in = c->rays[(k + c->ray_flip) & 1];
    b.out = c->rays[(k + 1 + c->ray_flip) & 1];
    b.n_in = c->ctr + C_RAYS + k;
    if (k == 0 && !rev) {
        b.gen_dirs = c->dirs;
        b.gen_src = c->f_tx;
        b.gen_N = c->cfg.rays_per_tx;
    }
    b.n_out = c->ctr + C_RAYS + k + 1;
    b.work = (unsigned int*)(c->ctr + C_WORK + k);
    if (c->dbg_on && !rev) {
        b.dbg_sel = c->dbg_sel;
        b.dbg_log = c->dbg_log;
        b.dbg_n = c->dbg_n;
        b.dbg_cap = EMRT_CAPTURE_LOG_ROWS;
    }
    return b;
}

// ---- rebuild-on-degradation of the moving objects' tree (Section III-A:
// between rediscoveries only parts of the scene change).  Refitting keeps
// the tree's topology while the objects move, so its boxes loosen; its
// quality (summed child box areas over the root's) is read back after every
// update, and a discovery frame rebuilds once the last known quality exceeds
// dyn_rebuild_ratio times the quality the last build had.  A read-back that
// has not completed, no known build quality, a ratio of 0, batched steps and
// steps under stream capture all rebuild, as before.
static bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

static void dy_quality_collect(emrt_ctx* c) {
    if (!c->dyq_pending || hipEventQuery(c->ev_dyq) != hipSuccess) return;
    c->dyq_pending = false;
    const double q = c->dyq_host[1] > 0.0 ? c->dyq_host[0] / c->dyq_host[1] : 0.0;
    c->dyq_last = q;
    if (c->dyq_pending_build) c->dyq_built = q;
}

static bool dy_rebuild_due(emrt_ctx* c) {
    if (c->batched || !(c->cfg.dyn_rebuild_ratio > 0.0) || capturing(c->stream)) return true;
    dy_quality_collect(c);
    if (c->dyq_pending || !(c->dyq_built > 0.0) || !(c->dyq_last > 0.0)) return true;
    return c->dyq_last > c->dyq_built * c->cfg.dyn_rebuild_ratio;
}

static void dy_quality_readback(emrt_ctx* c, bool built) {
    if (c->batched || !(c->cfg.dyn_rebuild_ratio > 0.0) || capturing(c->stream)) return;
    if (!c->dyq_host) {
        if (hipHostMalloc((void**)&c->dyq_host, 2 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            c->dyq_host = nullptr;
            return;
        }
        if (hipEventCreateWithFlags(&c->ev_dyq, hipEventDisableTiming) != hipSuccess) {
            c->ev_dyq = nullptr;
            return;
        }
    }
    if (!c->ev_dyq) return;
    tree_quality(c->dy, c->dyq_dev, c->stream);
    if (hipMemcpyAsync(c->dyq_host, c->dyq_dev, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipEventRecord(c->ev_dyq, c->stream) != hipSuccess)
        return;
    c->dyq_pending = true;
    c->dyq_pending_build = built;
}

// after the step's last kernel: the quality of the tree this step updated
static void step_finish(emrt_ctx* c) {
    if (c->dy_updated) dy_quality_readback(c, c->dy_updated_build);
    c->dy_updated = false;
}

static void step_pre(emrt_ctx* c, int discover) {
    hipStream_t st = c->stream;
    SceneDev& S = c->S;
    // counters: keep the cache sizes, clear the rest
    fill_u64(c->ctr + C_RAYS, 0ULL, C_NCACHE - C_RAYS, st);
    fill_u64(c->ctr + C_STATS, 0ULL, kNumCounters - C_STATS, st);
    fill_u32(c->flags, 0u, 16, st);  // device flags report this step only
    if (c->timing_on) {
        auto& set = c->evs[c->ev_parity];
        ev_flush(c, set);
        set.used = set.bounce_end = 0;
    }
    // end points that moved since the last step (all of them when there is none)
    endpoints_moved(c->f_tx, c->prev_tx, c->sz.n_tx, c->moved_tx, c->hist, st);
    endpoints_moved(c->f_rx, c->prev_rx, c->sz.n_rx, c->moved_rx, c->hist, st);
    // ---- frame geometry (Section II-A: BVH updated between frames)
    scene_world(S, c->f_xf, c->flags, st);
    scene_planes(S, st);
    scene_face_tv(S, st);
    // capture trees: only the bounce kernel reads them, so cached frames skip them
    const bool rev = discover && c->rev_n > 0;
    bool diff = c->cfg.diffraction && S.E > 0;
    const bool build_dy = S.T_d > 0 && (c->dy.n != S.T_d || (discover && dy_rebuild_due(c)));
    BuildJob jobs[3];
    int nj = 0;
    if (S.T_d > 0) tri_boxes(S, S.tris_dynamic, S.T_d, c->box_dy, st);
    if (build_dy) jobs[nj++] = BuildJob{c->box_dy, S.T_d, &c->dy};
    if (discover && !rev) {  // spheres on the receivers
        rx_boxes(c->f_rx, c->sz.n_rx, c->box_rx, st);
        jobs[nj++] = BuildJob{c->box_rx, c->sz.n_rx, &c->rxt};
    }
    if (rev) {  // spheres on the transmitters
        rx_boxes(c->f_tx, c->sz.n_tx, c->box_tx, st);
        jobs[nj++] = BuildJob{c->box_tx, c->sz.n_tx, &c->txt};
    }
    if (diff && discover && S.E_dyn > 0) {
        edge_boxes(S, S.edges_dynamic, S.E_dyn, c->box_ed, st);
        jobs[nj++] = BuildJob{c->box_ed, S.E_dyn, &c->etd};
    }
    bvh_build_many(jobs, nj, c->tmp, st);  // the frame's rebuilt trees, in one batch
    if (S.T_d > 0 && !build_dy) bvh_refit(c->box_dy, c->dy, st);
    if (build_dy && !c->batched) {
        c->dyn_rebuilds++;
        c->dyq_built = 0.0;  // known once this build's quality is read back
    }
    c->dy_updated = S.T_d > 1 && !c->batched;  // its quality is read back at the end of the step
    c->dy_updated_build = build_dy;
    if (S.T_d > 0) tri_prims(S, S.tris_dynamic, c->dy, c->dy_prims, st);
    if (discover && !rev) rx_prims(c->f_rx, c->rxt, c->rx_prims, st);
    if (rev) rx_prims(c->f_tx, c->txt, c->tx_prims, st);
    if (diff && discover && S.E_dyn > 0) edge_prims(S, S.edges_dynamic, c->etd, c->edge_prims + 2LL * S.E_s, st);
    if (discover) {
        KeySrc src = key_src(c, c->cache[c->cur]);
        const unsigned long long mask = (unsigned long long)c->table_slots - 1ULL;
        const int n_src = rev ? c->rev_n : c->sz.n_tx;
        fill_u64(c->table, 0ULL, c->table_slots, st);
        if (!rev) fill_u64(c->dbg_n, 0ULL, 1, st);  // the capture log holds the last transmitter-side discovery
        if (diff) fill_u32(c->illum, 0u, (long long)n_src * c->e_words, st);
        if (diff && c->pairs) fill_u64(c->pairs, 0ULL, c->pair_slots, st);
        cache_insert(c->table, mask, c->cache[c->cur], c->ctr + C_NCACHE + c->cur, c->P, src, c->flags, st);
        if (rev) {
            gather_rx(c->f_rx, c->rev_rx, c->rev_n, c->rev_pos, st);
            raygen(c->rev_pos, c->rev_n, c->rev_rays, nullptr, c->rays[0], c->ctr + C_RAYS, st);
        } else {
            // the primary rays are made by the first bounce launch (bounce_args)
            fill_u64(c->ctr + C_RAYS, (unsigned long long)c->n_total, 1, st);
        }
    }
}

static void step_bounces(emrt_ctx* c, bool fork_diff = false) {
    long long g = (launch_total(c) + 255) / 256;
    int grid = (int)std::min<long long>(std::max<long long>(g, 1), 2048);
    c->ray_flip = 0;
    c->regroup_now = true;
    for (int k = 0; k <= c->K; k++) {
        BounceArgs b = bounce_args(c, k, c->cur);
        ev_record(c);
        bounce(b, c->stats_on != 0, grid, c->stream);
        ev_record(c);
        if (b.out_key) {  // the next bounce's rays, grouped by origin cell and direction
            regroup(b.out, b.in, c->ray_key, c->ctr + C_RAYS + k + 1, c->n_total, c->rg_temp, c->stream);
            c->ray_flip ^= 1;
        }
        if (k == 0 && fork_diff) {
            // the edges lit by the first segments are known: candidates on the side stream
            HC(hipEventRecord(c->ev_fork, c->stream));
            HC(hipStreamWaitEvent(c->side, c->ev_fork, 0));
            const unsigned long long mask = (unsigned long long)c->table_slots - 1ULL;
            rx_grid_build(c->f_rx, c->sz.n_rx, c->bins, c->side);
            diff_candidates(path_args(c), c->illum, c->e_words, c->bins, c->table, mask, key_src(c, c->cache[c->cur]),
                            fresh_keys(c), c->side);
            HC(hipEventRecord(c->ev_join, c->side));
            c->diff_async = true;
        }
    }
    c->evs[c->ev_parity].bounce_end = c->evs[c->ev_parity].used;
    c->ray_flip = 0;
    c->regroup_now = false;
}

static void step_post(emrt_ctx* c, int discover) {
    hipStream_t st = c->stream;
    SceneDev& S = c->S;
    bool diff = c->cfg.diffraction && S.E > 0;
    KeySrc src = key_src(c, c->cache[c->cur]);
    PathArgs pa = path_args(c);
    const unsigned long long mask = (unsigned long long)c->table_slots - 1ULL;
    if (discover) {
        if (diff && c->rev_n > 0) {
            diff_candidates_rx(pa, c->illum, c->e_words, c->rev_rx, c->rev_n, c->table, mask, src, st);
        } else if (diff && c->diff_async) {  // launched beside the bounces
            HC(hipStreamWaitEvent(st, c->ev_join, 0));
            c->diff_async = false;
        } else if (diff) {
            rx_grid_build(c->f_rx, c->sz.n_rx, c->bins, st);
            diff_candidates(pa, c->illum, c->e_words, c->bins, c->table, mask, src, fresh_keys(c), st);
        }
        if (diff && c->pairs) {  // one reflection and one diffraction
            ExtraKeys xk{c->extra, c->ctr + C_NEXTRA, c->P};
            pair_candidates(pa, c->pairs, c->pair_slots, c->pair_list, c->ctr + C_NPAIRS, c->bins,
                            c->rev_n > 0 ? c->rev_rx : nullptr, xk, c->table, mask, src, st);
        }
        table_compact(c->table, (unsigned long long)c->table_slots, src, c->cand, c->ctr + C_NCAND, c->P, c->flags,
                      c->ctmp, st);
        cache_append(c->cache[c->cur], c->ctr + C_NCACHE + c->cur, c->P, c->ctr + C_NCAND, c->cand, c->P, c->flags, st);
        if (diff && c->rev_n == 0) fresh_append(fresh_keys(c), c->ctr + C_NCAND, c->cand, c->P, src, c->flags, st);
        pa.cand = c->cand;
        pa.n_cand = c->ctr + C_NCAND;
        c->discovered = true;
        c->last_rev = c->rev_n > 0;
    } else {
        pa.cand = c->cache[c->cur];
        pa.n_cand = c->ctr + C_NCACHE + c->cur;
        pa.cand_cached = 1;
    }
    // ---- exact validation + fields (Sections II-A, III-B, III-C)
    ev_record(c);
    validate_eval(pa, c->n_links, c->P, c->vtmp, st);
    ev_record(c);
    // ---- per-link reduction (Section V-D statistics)
    link_group(c->vp, c->sz.n_rx, c->n_links, c->link_cnt, c->link_off, c->scan_tmp, c->link_start, c->link_end,
               c->sv0, st);
    link_rank(c->vp, c->sz.n_rx, c->sv0, c->link_start, c->link_end, c->sv1, st);
    c->order = c->sv1;
    link_reduce(c->vp, c->order, c->link_start, c->link_end, c->n_links, c->nf, c->cfg.tx_power_w, c->chan, st);
    // ---- coherence statistics over frames (Section III-B)
    coherence_update(c->coh, c->vp, c->order, c->link_start, c->link_end, c->chan, c->n_links, c->nf, st);
    // ---- next cache: valid non-LoS keys in link/key order
    int nxt = 1 - c->cur;
    cache_counts(c->vp, c->order, c->link_start, c->link_end, c->n_links, c->link_cnt, st);
    exclusive_scan(c->link_cnt, c->link_off, c->n_links, c->scan_tmp, (uint32_t*)(c->ctr + C_NCACHE + nxt), st);
    fill_u32(((uint32_t*)(c->ctr + C_NCACHE + nxt)) + 1, 0u, 1, st);  // high word of the u64 count
    cache_write(c->vp, c->order, c->link_start, c->link_end, c->link_off, c->n_links, c->cache[nxt], st);
    fill_u32(c->hist, 1u, 1, st);  // the cache, end points and line-of-sight tests now belong together
    c->cur = nxt;
    c->stepped = true;
    c->frame_since_step = false;
    if (c->timing_on) {
        c->evs[c->ev_parity].pending = true;
        c->ev_parity ^= 1;
    }
}

int32_t emrt_step(emrt_ctx* c, int32_t discover) {
    if (!c) return EMRT_E_INVALID;
    if (!c->scene_set || !c->frame_set) return fail(c, EMRT_E_STATE, "set_scene and set_frame first");
    if (c->batched) return fail(c, EMRT_E_STATE, "context belongs to a batch: use emrt_batch_step");
    step_pre(c, discover);
    if (discover) {
        const bool fork = c->cfg.diffraction && c->S.E > 0 && c->K >= 1;
        if (fork && !c->side) {
            if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess)
                return fail(c, EMRT_E_HIP, "side stream");
        }
        step_bounces(c, fork);
    }
    step_post(c, discover);
    step_finish(c);
    return hip_check(c, hipGetLastError(), "step");
}

int32_t emrt_step_rx(emrt_ctx* c, const int32_t* rx_ids, int32_t n_src, int32_t rays_per_rx) {
    if (!c) return EMRT_E_INVALID;
    if (!c->scene_set || !c->frame_set) return fail(c, EMRT_E_STATE, "set_scene and set_frame first");
    if (c->batched) return fail(c, EMRT_E_STATE, "context belongs to a batch: use emrt_batch_step");
    if (!rx_ids || n_src < 1 || n_src > kMaxRxSources) return fail(c, EMRT_E_INVALID, "1..1024 receivers per launch");
    if (rays_per_rx < 1 || (long long)n_src * rays_per_rx > c->n_total)
        return fail(c, EMRT_E_INVALID, "receivers x rays_per_rx exceeds n_tx x rays_per_tx (the ray buffers)");
    for (int i = 0; i < n_src; i++)
        if (rx_ids[i] < 0 || rx_ids[i] >= c->sz.n_rx) return fail(c, EMRT_E_INVALID, "receiver index out of range");
    c->rev_host.assign(rx_ids, rx_ids + n_src);
    HC(hipMemcpyAsync(c->rev_rx, c->rev_host.data(), sizeof(int) * n_src, hipMemcpyHostToDevice, c->stream));
    c->rev_n = n_src;
    c->rev_rays = rays_per_rx;
    step_pre(c, 1);
    step_bounces(c);
    step_post(c, 1);
    step_finish(c);
    c->rev_n = 0;
    c->rev_rays = 0;
    return hip_check(c, hipGetLastError(), "step_rx");
}

int32_t emrt_backward(emrt_ctx* c, const double* dL_dH, const double* dL_dP, double* grad_eps, double* grad_tx_pos,
                      double* grad_tx_orient) {
    if (!c) return EMRT_E_INVALID;
    if (!c->stepped || c->frame_since_step)
        return fail(c, EMRT_E_STATE, "backward needs a step after the last set_frame");
    if (c->cfg.adjoint_materials <= 0 || !c->adj_rows)
        return fail(c, EMRT_E_UNSUPPORTED, "adjoint_materials is 0 in the configuration");
    if (c->S.M > c->cfg.adjoint_materials)
        return fail(c, EMRT_E_UNSUPPORTED, "more materials than adjoint_materials");
    AdjArgs a{};
    a.s = c->S;
    a.fc.mat_eps = c->mat;
    a.fc.mat_refl = c->refl;
    a.fc.nf = c->nf;
    for (int i = 0; i < EMRT_NF; i++) a.fc.freq[i] = i < c->nf ? c->cfg.freq_hz[i] : 1.0;
    a.fc.ant_mode = c->cfg.antenna_mode;
    a.tx_pos = c->f_tx;
    a.tx_orient = c->f_txo;
    a.rx_pos = c->f_rx;
    a.vp = c->vp;
    a.order = c->order;
    a.start = c->link_start;
    a.end = c->link_end;
    a.chan = c->chan;
    a.dL_dH = dL_dH;
    a.dL_dP = dL_dP;
    a.p_tx = c->cfg.tx_power_w;
    a.n_links = c->n_links;
    a.M = c->S.M;
    a.combined = c->cfg.diffraction == 2 ? 1 : 0;
    a.rows = c->adj_rows;
    a.n_rx = c->sz.n_rx;
    a.path_tan = (double*)c->leg_block;
    a.path_eps = a.path_tan + 5LL * c->vcap;
    adjoint(a, c->sz.n_tx, c->sz.n_rx, grad_tx_pos, grad_tx_orient, grad_eps, c->stream);
    return hip_check(c, hipGetLastError(), "backward");
}

int32_t emrt_read_coherence(emrt_ctx* c, double R, const emrt_coherence_view* v, double* min_tc,
                            int64_t* n_triggered) {
    if (!c || !v) return EMRT_E_INVALID;
    if (!(R > 0.0 && R < 1.0)) return fail(c, EMRT_E_INVALID, "correlation threshold R must be in (0, 1)");
    if (!c->stepped) return fail(c, EMRT_E_STATE, "no step yet");
    unsigned long long* tmp = c->ctr + C_COH;  // [2] min_tc bits, triggered count
    unsigned long long init[2] = {0x7FF0000000000000ULL, 0ULL};  // +inf, 0
    HC(hipMemcpyAsync(tmp, init, sizeof(init), hipMemcpyHostToDevice, c->stream));
    CohRead r{R, v->tc, v->corr, v->trigger, tmp, tmp + 1};
    FieldCtx fc{};
    fc.nf = c->nf;
    for (int i = 0; i < EMRT_NF; i++) fc.freq[i] = i < c->nf ? c->cfg.freq_hz[i] : 1.0;
    coherence_read(c->coh, r, c->n_links, c->sz.n_rx, c->nf, c->f_tx, c->f_txv, c->f_rx, c->f_rxv, fc, c->stream);
    unsigned long long h[2];
    int32_t rc = sync_read(c, h, tmp, sizeof(h));
    if (rc) return rc;
    if (min_tc) memcpy(min_tc, &h[0], sizeof(double));
    if (n_triggered) *n_triggered = (int64_t)h[1];
    return emrt_sync(c);
}

int32_t emrt_coherence_reset(emrt_ctx* c) {
    if (!c) return EMRT_E_INVALID;
    if (!c->bound) return fail(c, EMRT_E_STATE, "no workspace");
    coherence_clear(c);
    return hip_check(c, hipGetLastError(), "coherence_reset");
}

int32_t emrt_sync(emrt_ctx* c) {
    if (!c) return EMRT_E_INVALID;
    uint32_t fl = 0;
    if (c->bound) {
        int32_t rc = sync_read(c, &fl, c->flags, sizeof(fl));
        if (rc) return rc;
    } else {
        return hip_check(c, hipStreamSynchronize(c->stream), "sync");
    }
    c->flag_accum |= fl;
    if (fl & (FLAG_BAD_INPUT | FLAG_NONFINITE)) return fail(c, EMRT_E_DEVICE_FLAG, "non-finite or invalid frame input");
    if (fl & (FLAG_TABLE_FULL | FLAG_CAND_CAP | FLAG_PATH_CAP))
        return fail(c, EMRT_W_CACHE_FULL, "capacity reached (path table, candidates or paths): results incomplete");
    return EMRT_OK;
}

}  // extern "C"

// channel copy into caller layout
__global__ void k_read_channels(const double* chan, long long n_links, int nf, double* H, double* Pc, double* Pi,
                                double* tm, double* tr, double* fm, double* fr, int32_t* np, uint32_t* fl) {
    long long n = n_links * nf;
    const int* ci = (const int*)(chan + 8 * n);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const double* c = chan + 8 * i;
        if (H) { H[2 * i] = c[0]; H[2 * i + 1] = c[1]; }
        if (Pc) Pc[i] = c[2];
        if (Pi) Pi[i] = c[3];
        if (tm) tm[i] = c[4];
        if (tr) tr[i] = c[5];
        if (fm) fm[i] = c[6];
        if (fr) fr[i] = c[7];
        if (i < n_links) {
            if (np) np[i] = ci[2 * i];
            if (fl) fl[i] = ci[2 * i + 1] ? 1u : 0u;
        }
    }
}

__global__ void k_trunc_flag(const int* start, const int* end, long long n_links, int cap, unsigned long long* flag) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_links; i += (long long)gridDim.x * blockDim.x) {
        if (start[i] >= 0 && end[i] - start[i] > cap) atomicOr(flag, 1ULL);
    }
}

extern "C" {

int32_t emrt_read_channels(emrt_ctx* c, const emrt_channel_view* v) {
    if (!c || !v) return EMRT_E_INVALID;
    if (!c->stepped) return fail(c, EMRT_E_STATE, "no step yet");
    long long n = c->n_links * c->nf;
    int g = (int)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_read_channels, dim3(std::max(g, 1)), dim3(256), 0, c->stream, c->chan, c->n_links, c->nf,
                       v->H, v->P_coh, v->P_inc, v->tau_mean, v->tau_rms, v->fd_mean, v->fd_rms, v->n_paths,
                       v->flags);
    return emrt_sync(c);
}

int32_t emrt_read_paths(emrt_ctx* c, const emrt_path_view* v) {
    if (!c || !v || v->cap < 1 || !v->count) return fail(c, EMRT_E_INVALID, "bad path view");
    if (!c->stepped) return fail(c, EMRT_E_STATE, "no step yet");
    path_gather(c->vp, c->order, c->link_start, c->link_end, c->n_links, c->nf, v->cap, v->key, v->tri_ids, v->a,
                v->tau, v->fd, v->angles, v->count, c->stream);
    fill_u64(c->ctr + C_TRUNC, 0ULL, 1, c->stream);
    int g = (int)std::min<long long>((c->n_links + 255) / 256, 4096);
    hipLaunchKernelGGL(k_trunc_flag, dim3(std::max(g, 1)), dim3(256), 0, c->stream, c->link_start, c->link_end,
                       c->n_links, v->cap, c->ctr + C_TRUNC);
    unsigned long long tr = 0;
    int32_t rc = sync_read(c, &tr, c->ctr + C_TRUNC, sizeof(tr));
    if (rc) return rc;
    rc = emrt_sync(c);
    if (rc) return rc;
    return tr ? EMRT_W_PATHS_TRUNCATED : EMRT_OK;
}

int32_t emrt_debug_ray_records(emrt_ctx* c, int32_t tx, const int32_t* ray_ids, int32_t n, int32_t* out) {
    if (!c || (n > 0 && (!ray_ids || !out)) || tx < 0 || tx >= c->sz.n_tx) return fail(c, EMRT_E_INVALID, "bad arguments");
    if (!c->discovered) return fail(c, EMRT_E_STATE, "no discovery step yet");
    if (c->last_rev) return fail(c, EMRT_E_STATE, "the last discovery step launched from receivers");
    debug_rays(c->hitlog, c->depth, c->n_total, c->K, tx, c->cfg.rays_per_tx, c->dir_slot, ray_ids, n, out,
               c->stream);
    return hip_check(c, hipGetLastError(), "debug_ray_records");
}

int32_t emrt_debug_select_rays(emrt_ctx* c, int32_t tx, const int32_t* ray_ids, int32_t n) {
    if (!c || n < 0 || (n > 0 && !ray_ids) || tx < 0 || tx >= c->sz.n_tx) return fail(c, EMRT_E_INVALID, "bad arguments");
    if (!c->scene_set) return fail(c, EMRT_E_STATE, "set_scene first");
    if (n == 0) {
        fill_u32(c->dbg_sel, 0u, c->n_total / 32 + 1, c->stream);
        c->dbg_on = false;
        return hip_check(c, hipGetLastError(), "debug_select_rays");
    }
    uint32_t* bad = (uint32_t*)(c->ctr + C_SCRATCH);
    fill_u32(bad, 0u, 1, c->stream);
    debug_mark(c->dbg_sel, tx, c->cfg.rays_per_tx, c->dir_slot, ray_ids, n, bad, c->stream);
    uint32_t h = 0;
    int32_t rc = sync_read(c, &h, bad, sizeof(h));
    if (rc) return rc;
    c->dbg_on = true;
    return h ? fail(c, EMRT_E_INVALID, "launch direction outside [0, rays_per_tx)") : EMRT_OK;
}

int32_t emrt_debug_ray_captures(emrt_ctx* c, int32_t* out, int64_t cap, int64_t* n_rows) {
    if (!c || !n_rows || cap < 0 || (cap > 0 && !out)) return fail(c, EMRT_E_INVALID, "bad arguments");
    if (!c->bound) return fail(c, EMRT_E_STATE, "no workspace");
    if (cap > 0)
        debug_captures(c->dbg_log, c->dbg_n, EMRT_CAPTURE_LOG_ROWS, c->cfg.rays_per_tx, c->dir_perm, out, cap,
                       c->stream);
    unsigned long long n = 0;
    int32_t rc = sync_read(c, &n, c->dbg_n, sizeof(n));
    if (rc) return rc;
    const unsigned long long kept = std::min<unsigned long long>(n, (unsigned long long)EMRT_CAPTURE_LOG_ROWS);
    *n_rows = (int64_t)std::min<unsigned long long>(kept, (unsigned long long)cap);
    return n > (unsigned long long)*n_rows ? EMRT_W_PATHS_TRUNCATED : EMRT_OK;
}

int32_t emrt_cache_size(emrt_ctx* c, int64_t* n) {
    if (!c || !n) return EMRT_E_INVALID;
    if (!c->bound) return fail(c, EMRT_E_STATE, "no workspace");
    unsigned long long v = 0;
    int32_t rc = sync_read(c, &v, c->ctr + C_NCACHE + c->cur, sizeof(v));
    *n = (int64_t)std::min<unsigned long long>(v, (unsigned long long)c->P);
    return rc;
}

int32_t emrt_cache_export(emrt_ctx* c, int32_t* keys, int64_t cap, int64_t* n) {
    if (!c || !n) return EMRT_E_INVALID;
    int64_t m = 0;
    int32_t rc = emrt_cache_size(c, &m);
    if (rc) return rc;
    *n = m;
    if (m > cap) return fail(c, EMRT_E_INVALID, "export buffer too small");
    if (m > 0 && !keys) return fail(c, EMRT_E_INVALID, "null export buffer");
    keys_export(c->cache[c->cur], m, keys, c->stream);
    return hip_check(c, hipStreamSynchronize(c->stream), "cache_export");
}

int32_t emrt_cache_import(emrt_ctx* c, const int32_t* keys, int64_t n) {
    if (!c || n < 0 || (n > 0 && !keys)) return EMRT_E_INVALID;
    if (!c->scene_set) return fail(c, EMRT_E_STATE, "set_scene first");
    if (n > c->P) return fail(c, EMRT_E_INVALID, "more keys than path_capacity");
    keys_import(keys, n, c->cache[c->cur], c->stream);
    fill_u32(c->hist, 0u, 1, c->stream);  // imported keys were not validated here
    unsigned long long v = (unsigned long long)n;
    HC(hipMemcpyAsync(c->ctr + C_NCACHE + c->cur, &v, sizeof(v), hipMemcpyHostToDevice, c->stream));
    return hip_check(c, hipStreamSynchronize(c->stream), "cache_import");
}

int32_t emrt_read_stats(emrt_ctx* c, emrt_stats* o) {
    if (!c || !o) return EMRT_E_INVALID;
    if (!c->bound) return fail(c, EMRT_E_STATE, "no workspace");
    unsigned long long h[kNumCounters];
    int32_t rc = sync_read(c, h, c->ctr, sizeof(h));
    if (rc) return rc;
    uint32_t fl = 0;
    if ((rc = sync_read(c, &fl, c->flags, sizeof(fl)))) return rc;
    memset(o, 0, sizeof(*o));
    for (int b = 0; b < 7; b++) o->rays_per_bounce[b] = b <= c->K ? (int64_t)h[C_RAYS + b] : 0;
    o->n_candidates = (int64_t)h[C_NCAND];
    o->n_valid = (int64_t)h[C_NVALID];
    o->n_cache = (int64_t)h[C_NCACHE + c->cur];
    o->node_visits = (int64_t)h[C_STATS + 0];
    o->tri_tests = (int64_t)h[C_STATS + 1];
    o->segments = (int64_t)h[C_STATS + 2];
    o->captures = (int64_t)h[C_STATS + 3];
    o->wide_box_tests = (int64_t)h[C_STATS + 16];
    o->n_static_tris = c->S.T_s;
    o->n_dynamic_tris = c->S.T_d;
    o->n_edges = c->S.E;
    o->device_flags = fl | c->flag_accum;
    for (auto& set : c->evs) ev_flush(c, set);
    o->bounce_ms = c->t_bounce_ms;
    o->bounce_launches = c->t_bounce_n;
    o->validate_ms = c->t_validate_ms;
    o->validate_launches = c->t_validate_n;
    o->static_tree_area = c->st_area;
    dy_quality_collect(c);
    o->dyn_rebuilds = c->dyn_rebuilds;
    o->dyn_tree_quality = c->dyq_last;
    return EMRT_OK;
}

const char* emrt_status_string(int32_t s) {
    switch (s) {
        case EMRT_OK: return "ok";
        case EMRT_W_PATHS_TRUNCATED: return "warning: path list truncated";
        case EMRT_W_CACHE_FULL: return "warning: capacity reached, results incomplete";
        case EMRT_E_INVALID: return "invalid argument";
        case EMRT_E_STATE: return "call out of order";
        case EMRT_E_WORKSPACE: return "workspace missing or too small";
        case EMRT_E_HIP: return "HIP error";
        case EMRT_E_UNSUPPORTED: return "unsupported configuration";
        case EMRT_E_DEVICE_FLAG: return "device reported invalid input";
        default: return "unknown status";
    }
}

int32_t emrt_last_error(emrt_ctx* c, char* buf, size_t len) {
    if (!c || !buf || len == 0) return EMRT_E_INVALID;
    size_t n = std::min(len - 1, c->err.size());
    memcpy(buf, c->err.data(), n);
    buf[n] = 0;
    return EMRT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batch ----
// Batched stepping of several independent scenes (each a context with its
// own workspace): the per-scene phases run on n_streams streams (scenes
// round-robin), the bounces of all scenes run as one persistent launch per
// bounce level (k_bounce_multi over a device table of chunk offsets), and
// the whole step is captured once per (discover, cache parity) as a HIP graph
// and replayed.  Results are those of stepping each context alone.
struct emrt_batch {
    std::vector<emrt_ctx*> ctx;
    std::vector<hipStream_t> own_stream;  // each member's stream before the batch took it over
    int kmax = 0;
    hipStream_t stream = nullptr;
    std::vector<hipStream_t> side;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    int n_streams = 4, grid = 2048, chunk = 64;
    bool use_graph = true;
    // workspace
    char* ws = nullptr;
    BounceArgs* args = nullptr;  // [2 parities][kmax + 1][n]
    uint32_t* chunk_off = nullptr;  // [kmax + 1][n + 1]
    uint32_t* work = nullptr;       // [kmax + 1]
    unsigned long long* zero = nullptr;
    bool args_ready[2] = {false, false};
    hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [discover][parity]
    std::string err;
};

static size_t batch_layout(emrt_batch* b, Carver& cv) {
    long long n = (long long)b->ctx.size();
    b->args = cv.take<BounceArgs>(2LL * (b->kmax + 1) * n);
    b->chunk_off = cv.take<uint32_t>((long long)(b->kmax + 1) * (n + 1));
    b->work = cv.take<uint32_t>(b->kmax + 1);
    b->zero = cv.take<unsigned long long>(1);
    return cv.off;
}

static void batch_drop_graphs(emrt_batch* b) {
    for (auto& row : b->exec)
        for (auto& e : row)
            if (e) {
                (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
}

static void batch_streams(emrt_batch* b) {
    for (auto s : b->side) (void)hipStreamDestroy(s);
    b->side.clear();
    for (auto e : b->join) (void)hipEventDestroy(e);
    b->join.clear();
    for (int i = 0; i + 1 < b->n_streams; i++) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) break;
        b->side.push_back(s);
        hipEvent_t e;
        (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
        b->join.push_back(e);
    }
}

// run f(ctx) for every scene, scene i on stream i mod (1 + side streams)
template <class F>
static void batch_fan(emrt_batch* b, F f) {
    int ns = 1 + (int)b->side.size();
    if (ns > 1) {
        (void)hipEventRecord(b->fork, b->stream);
        for (auto s : b->side) (void)hipStreamWaitEvent(s, b->fork, 0);
    }
    for (size_t i = 0; i < b->ctx.size(); i++) {
        int k = (int)(i % ns);
        b->ctx[i]->stream = k == 0 ? b->stream : b->side[k - 1];
        f(b->ctx[i]);
    }
    for (size_t j = 0; j < b->side.size(); j++) {
        (void)hipEventRecord(b->join[j], b->side[j]);
        (void)hipStreamWaitEvent(b->stream, b->join[j], 0);
    }
    for (auto c : b->ctx) c->stream = b->stream;
}

static void batch_enqueue(emrt_batch* b, int discover, int parity) {
    batch_fan(b, [&](emrt_ctx* c) { step_pre(c, discover); });
    if (discover) {
        long long n = (long long)b->ctx.size();
        // rays per chunk by level: the primary rays (level 0, the most and the
        // most coherent) twice the set chunk, at most 1024; level 1 the set
        // chunk; the later levels, with fewer rays, at most 256 (a shorter
        // tail).  On 64 uneven cities at chunk 512: 32.7-35.2 ms per step
        // against 35.3-37.2 with 512 at level 0, and 36.1 against 38.7-39.3
        // with 512 at every level.
        for (int k = 0; k <= b->kmax; k++) {
            const int ch = k == 0 ? std::min(2 * b->chunk, 1024) : (k == 1 ? b->chunk : std::min(b->chunk, 256));
            bounce_multi(b->args + ((long long)parity * (b->kmax + 1) + k) * n, (int)n,
                         b->chunk_off + (long long)k * (n + 1), b->work + k, b->grid, ch, b->stream);
        }
    }
    batch_fan(b, [&](emrt_ctx* c) { step_post(c, discover); });
}

static int32_t batch_fail(emrt_batch* b, int32_t st, const std::string& m) {
    if (b) b->err = m;
    return st;
}

extern "C" {

int32_t emrt_batch_create(emrt_ctx* const* ctxs, int32_t n, emrt_batch** out) {
    if (!ctxs || n < 1 || !out) return EMRT_E_INVALID;
    *out = nullptr;
    emrt_batch* b = new emrt_batch();
    for (int i = 0; i < n; i++) {
        emrt_ctx* c = ctxs[i];
        if (!c || !c->bound || !c->scene_set || c->batched) {
            delete b;
            return EMRT_E_STATE;
        }
        for (int j = 0; j < i; j++)
            if (ctxs[j] == c) {
                delete b;
                return EMRT_E_INVALID;
            }
        b->ctx.push_back(c);
        b->own_stream.push_back(c->stream);
        b->kmax = std::max(b->kmax, c->K);
    }
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return EMRT_E_HIP;
    }
    b->stream = ctxs[0]->stream;
    batch_streams(b);
    for (auto c : b->ctx) {
        c->batched = true;
        c->stream = b->stream;
    }
    *out = b;
    return EMRT_OK;
}

int32_t emrt_batch_destroy(emrt_batch* b) {
    if (!b) return EMRT_E_INVALID;
    (void)hipStreamSynchronize(b->stream);
    batch_drop_graphs(b);
    for (auto s : b->side) (void)hipStreamSynchronize(s);
    for (auto s : b->side) (void)hipStreamDestroy(s);
    for (auto e : b->join) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    // members go back to their own streams: the batch stream belongs to the
    // batch's caller and may be destroyed with it
    for (size_t i = 0; i < b->ctx.size(); i++) {
        b->ctx[i]->batched = false;
        b->ctx[i]->stream = b->own_stream[i];
    }
    delete b;
    return EMRT_OK;
}

int32_t emrt_batch_workspace_size(emrt_batch* b, size_t* bytes) {
    if (!b || !bytes) return EMRT_E_INVALID;
    Carver m(nullptr);
    *bytes = batch_layout(b, m) + 256;
    return EMRT_OK;
}

int32_t emrt_batch_bind_workspace(emrt_batch* b, void* ptr, size_t bytes) {
    if (!b || !ptr) return batch_fail(b, EMRT_E_WORKSPACE, "null workspace");
    Carver m(nullptr);
    char* base = (char*)(((uintptr_t)ptr + 255) & ~(uintptr_t)255);
    if (bytes < batch_layout(b, m) + (size_t)(base - (char*)ptr)) return batch_fail(b, EMRT_E_WORKSPACE, "too small");
    Carver cv(base);
    batch_layout(b, cv);
    b->ws = (char*)ptr;
    b->args_ready[0] = b->args_ready[1] = false;
    batch_drop_graphs(b);
    fill_u64(b->zero, 0ULL, 1, b->stream);
    return EMRT_OK;
}

int32_t emrt_batch_set_stream(emrt_batch* b, void* s) {
    if (!b) return EMRT_E_INVALID;
    b->stream = (hipStream_t)s;
    for (auto c : b->ctx) c->stream = b->stream;
    batch_drop_graphs(b);
    return EMRT_OK;
}

int32_t emrt_batch_set_options(emrt_batch* b, int32_t use_graph, int32_t n_streams, int32_t grid, int32_t chunk) {
    if (!b || n_streams < 1 || n_streams > 16 || grid < 1 || grid > (1 << 20)) return EMRT_E_INVALID;
    if (chunk != 32 && chunk != 64 && chunk != 128 && chunk != 256 && chunk != 512 && chunk != 1024)
        return EMRT_E_INVALID;
    (void)hipStreamSynchronize(b->stream);
    batch_drop_graphs(b);
    b->use_graph = use_graph != 0;
    b->grid = grid;
    b->chunk = chunk;
    if (n_streams != b->n_streams) {
        b->n_streams = n_streams;
        batch_streams(b);
    }
    return EMRT_OK;
}

int32_t emrt_batch_step(emrt_batch* b, int32_t discover) {
    if (!b) return EMRT_E_INVALID;
    if (!b->ws) return batch_fail(b, EMRT_E_WORKSPACE, "bind a batch workspace first");
    const int parity = b->ctx[0]->cur;
    for (auto c : b->ctx) {
        if (!c->scene_set || !c->frame_set) return batch_fail(b, EMRT_E_STATE, "set_scene and set_frame on every member");
        if (c->cur != parity) return batch_fail(b, EMRT_E_STATE, "members stepped separately");
    }
    discover = discover ? 1 : 0;
    const long long n = (long long)b->ctx.size();
    if (discover && !b->args_ready[parity]) {
        std::vector<BounceArgs> h((size_t)(b->kmax + 1) * n);
        for (int k = 0; k <= b->kmax; k++)
            for (long long i = 0; i < n; i++) {
                emrt_ctx* c = b->ctx[i];
                BounceArgs a = bounce_args(c, std::min(k, c->K), parity);
                if (k > c->K) a.n_in = b->zero;  // scene with fewer bounces: nothing to trace
                a.dbg_sel = nullptr;  // the capture log is a single-context tool (the table outlives marks)
                h[(size_t)k * n + i] = a;
            }
        BounceArgs* dst = b->args + (long long)parity * (b->kmax + 1) * n;
        hipError_t e = hipMemcpyAsync(dst, h.data(), sizeof(BounceArgs) * h.size(), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return batch_fail(b, EMRT_E_HIP, hipGetErrorString(e));
        b->args_ready[parity] = true;
    }
    // timing and statistics instrumentation is not used in batched steps
    std::vector<int> timing(n), stats(n);
    for (long long i = 0; i < n; i++) {
        timing[i] = b->ctx[i]->timing_on;
        stats[i] = b->ctx[i]->stats_on;
        b->ctx[i]->timing_on = 0;
        b->ctx[i]->stats_on = 0;
    }
    int32_t rc = EMRT_OK;
    if (!b->use_graph) {
        batch_enqueue(b, discover, parity);
    } else {
        hipGraphExec_t& ex = b->exec[discover][parity];
        if (!ex) {
            // capture: enqueueing advances host state, which the graph has not
            // executed yet; keep it and restore after the capture
            std::vector<int> cur(n);
            std::vector<char> disc(n);
            std::vector<int> dyn(n);
            for (long long i = 0; i < n; i++) {
                cur[i] = b->ctx[i]->cur;
                disc[i] = b->ctx[i]->discovered;
                dyn[i] = b->ctx[i]->dy.n;
            }
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed);
            if (e == hipSuccess) {
                batch_enqueue(b, discover, parity);
                e = hipStreamEndCapture(b->stream, &g);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            for (long long i = 0; i < n; i++) {
                b->ctx[i]->cur = cur[i];
                b->ctx[i]->discovered = disc[i];
                b->ctx[i]->dy.n = dyn[i];
            }
            if (e != hipSuccess) {
                ex = nullptr;
                rc = batch_fail(b, EMRT_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            }
        }
        if (rc == EMRT_OK) {
            hipError_t e = hipGraphLaunch(ex, b->stream);
            if (e != hipSuccess) rc = batch_fail(b, EMRT_E_HIP, std::string("graph launch: ") + hipGetErrorString(e));
            for (auto c : b->ctx) {
                c->cur = 1 - parity;
                if (discover) c->discovered = true;
                if (c->S.T_d > 0) c->dy.n = c->S.T_d;
            }
        }
    }
    for (long long i = 0; i < n; i++) {
        b->ctx[i]->timing_on = timing[i];
        b->ctx[i]->stats_on = stats[i];
        if (rc == EMRT_OK) {
            b->ctx[i]->stepped = true;
            b->ctx[i]->frame_since_step = false;
        }
    }
    if (rc != EMRT_OK) return rc;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? EMRT_OK : batch_fail(b, EMRT_E_HIP, hipGetErrorString(e));
}

// Autotune the launch shape on real discovery steps (the member frames as
// set): the persistent grid of the multi-scene bounce, then the number of
// streams the per-scene phases are spread over.  Each trial is one eager
// discovery step timed with HIP events on the batch stream.
int32_t emrt_batch_autotune(emrt_batch* b, int32_t repeats, int32_t* best_grid, int32_t* best_streams,
                            int32_t* best_chunk) {
    if (!b || repeats < 1 || repeats > 15) return EMRT_E_INVALID;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return batch_fail(b, EMRT_E_HIP, "event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return batch_fail(b, EMRT_E_HIP, "event");
    }
    const bool graph = b->use_graph;
    // one trial: `repeats` timed discovery steps (no graph: the options change
    // every trial), their median
    auto trial = [&](int grid, int ns, int chunk, int reps, float& med) -> int32_t {
        int32_t rc = emrt_batch_set_options(b, 0, ns, grid, chunk);
        if (rc) return rc;
        float t[15];
        for (int r = 0; r < reps; r++) {
            (void)hipEventRecord(e0, b->stream);
            rc = emrt_batch_step(b, 1);
            (void)hipEventRecord(e1, b->stream);
            if (rc) return rc;
            if (hipEventSynchronize(e1) != hipSuccess) return batch_fail(b, EMRT_E_HIP, "autotune sync");
            (void)hipEventElapsedTime(&t[r], e0, e1);
        }
        std::sort(t, t + reps);
        med = t[reps / 2];
        return EMRT_OK;
    };
    float warm = 0;
    int32_t rc = trial(b->grid, b->n_streams, b->chunk, 1, warm);  // first touch, code loading
    int g_best = b->grid, s_best = b->n_streams, c_best = b->chunk;
    float t_best = 1e30f;
    const int grids[] = {1024, 2048, 4096, 8192};
    const int streams[] = {1, 2, 4, 8};
    const int chunks[] = {64, 128, 256, 512};
    for (int ns : streams)
        for (int g : grids)
            for (int ch : chunks) {
                float ms = 0;
                if (rc == EMRT_OK) rc = trial(g, ns, ch, repeats, ms);
                if (rc == EMRT_OK && ms < t_best) {
                    t_best = ms;
                    g_best = g;
                    s_best = ns;
                    c_best = ch;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != EMRT_OK) return rc;
    rc = emrt_batch_set_options(b, graph ? 1 : 0, s_best, g_best, c_best);
    if (best_grid) *best_grid = g_best;
    if (best_streams) *best_streams = s_best;
    if (best_chunk) *best_chunk = c_best;
    return rc;
}

int32_t emrt_batch_sync(emrt_batch* b) {
    if (!b) return EMRT_E_INVALID;
    int32_t worst = EMRT_OK;
    for (auto c : b->ctx) {
        int32_t r = emrt_sync(c);
        if (r < 0 && (worst >= 0 || r < worst)) worst = r;
        else if (r > 0 && worst == EMRT_OK) worst = r;
    }
    return worst;
}

int32_t emrt_batch_last_error(emrt_batch* b, char* buf, size_t len) {
    if (!b || !buf || len == 0) return EMRT_E_INVALID;
    size_t k = std::min(len - 1, b->err.size());
    memcpy(buf, b->err.data(), k);
    buf[k] = 0;
    return EMRT_OK;
}

}  // extern "C"
