/*
 * emrt.h -- C ABI of the gfx950 dynamic EM ray tracer.
 *
 * The library implements the data-parallel hot path of Wang & Manocha,
 * "Dynamic EM Ray Tracing for Large Urban Scenes with Multiple Receivers"
 * (2023): shooting-and-bouncing rays from transmitters through LBVHs over
 * static buildings and moving vehicles (Section II-A: direct, reflected and
 * diffracted rays, a BVH updated between frames), receiver capture,
 * revalidation of cached paths across frames (Section III-B: the path cache /
 * "visibility hash table" with deletion), and per-receiver sums of complex
 * field, power, delay and Doppler (Section III-C Eq (3); Section V-D: mean
 * Doppler shift and RMS Doppler spread).
 *
 * Conventions
 *   - Every call returns an emrt status: EMRT_OK (0), a warning (> 0) or an
 *     error (< 0).  emrt_last_error() gives the message of the last error.
 *   - All work is enqueued on the context's HIP stream (emrt_set_stream).
 *     Calls return without waiting for the GPU unless their name contains
 *     "read", "sync", "size" or "export", or they are emrt_set_scene /
 *     emrt_cache_import (which read back counts).
 *   - Memory: the caller owns every buffer.  The library never allocates
 *     device memory: it carves one caller-allocated workspace
 *     (emrt_workspace_size / emrt_bind_workspace), or its own static array
 *     for callers that cannot allocate (emrt_bind_static_workspace).  Arrays marked "device"
 *     are device pointers read or written in stream order; the caller keeps
 *     them alive and unmodified until the stream has passed the call.
 *     Arrays marked "host" are copied before the call returns.
 *   - A context is used from one host thread at a time.
 *   - Positions in metres, velocities in m/s, frequencies in Hz, delays in s,
 *     powers in W; complex numbers are (re, im) double pairs; time factor
 *     exp(+j w t), permittivity eps_r = eps' - j eps'' (imaginary part <= 0).
 */
#ifndef EMRT_H
#define EMRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    EMRT_OK = 0,
    EMRT_W_PATHS_TRUNCATED = 1, /* a link had more paths than the path-list capacity */
    EMRT_W_CACHE_FULL = 2,      /* path table / candidate / path capacity reached: results incomplete */
    EMRT_E_INVALID = -1,        /* bad argument or malformed input */
    EMRT_E_STATE = -2,          /* call out of order (e.g. step before scene) */
    EMRT_E_WORKSPACE = -3,      /* workspace missing or too small */
    EMRT_E_HIP = -4,            /* HIP runtime error */
    EMRT_E_UNSUPPORTED = -5,    /* configuration outside the supported range */
    EMRT_E_DEVICE_FLAG = -6     /* a kernel reported bad input (non-finite transform, ...) */
};

enum { EMRT_ANT_ISO_V = 0, EMRT_ANT_DIPOLE = 1 };

typedef struct emrt_ctx emrt_ctx;

/* Configuration (host struct, copied by emrt_ctx_create).  Readings of the
 * paper (which fixes none of these): launch on a Fibonacci sphere,
 * reception-sphere radius k_rx * sqrt(4 pi / N) * unfolded length, no power
 * threshold, first-order edge diffraction for receivers within
 * diff_max_leg_m of the diffraction point. */
typedef struct emrt_config {
    int32_t n_freq;             /* 1..4 */
    double freq_hz[4];          /* carrier frequencies evaluated on the same paths */
    int32_t max_reflections;    /* K, 0..5 */
    int32_t diffraction;        /* 0: none; 1: first-order edge diffraction; 2 (one reflection with one
                                   diffraction: transmitter-side steps propose reflection then
                                   diffraction, receiver-side steps diffraction then reflection) is
                                   refused with EMRT_E_UNSUPPORTED for now */
    int32_t rays_per_tx;        /* N launch directions per transmitter, >= 1 */
    double rx_sphere_k;         /* reception-sphere constant k_rx (default 1.0) */
    double diff_max_leg_m;      /* max edge-to-receiver distance (default 250) */
    double tx_power_w;          /* transmit power (default 100 W = 50 dBm, Section IV) */
    int32_t antenna_mode;       /* transmit antenna: EMRT_ANT_ISO_V (Section IV) or EMRT_ANT_DIPOLE */
    int32_t path_cap_per_link;  /* default path-list capacity per link (emrt_read_paths) */
    int64_t path_capacity;      /* max candidate keys per frame and cached paths (default 4 Mi) */
    int64_t table_capacity;     /* path-table slots, rounded up to a power of two (default 4 x path_capacity) */
    int32_t adjoint_materials;  /* 0: no adjoint; else the most materials emrt_backward supports (<= 256);
                                   adds 8 (5 + 2 adjoint_materials) bytes per link to the workspace */
    double dyn_rebuild_ratio;   /* > 0: the tree over the moving objects' triangles is refitted on
                                   every frame and rebuilt on a discovery frame only once its quality
                                   (summed child box areas over the root's, read back one step late)
                                   exceeds this multiple of its value when last built (Section III-A:
                                   only what changed is rebuilt); 0 (default): rebuilt on every
                                   discovery frame, refitted on cached ones.  Batched steps always
                                   rebuild.  Results do not depend on the tree; a choice for scenes
                                   whose moving geometry is large (on the city's 24,000 vehicle
                                   triangles a rebuild costs less than a looser tree) */
    int32_t ray_regroup;        /* 1: the rays entering bounces 2..K are regrouped by origin cell and
                                   direction octant (one counting sort per bounce), so a wave traces
                                   neighbouring rays; 0 (default): they stay in the order the previous
                                   bounce appended them.  Results are the same either way.  On the
                                   2 x 2 km city the sorts cost more than the traversal gains (it is
                                   a choice for scenes with longer ray paths); adds 2 bytes per
                                   launched ray to the workspace */
} emrt_config;

/* Fill *cfg with the defaults above (one 28 GHz carrier, K = 3, no
 * diffraction, 10,000 rays per transmitter, no regrouping between bounces). */
void emrt_config_default(emrt_config* cfg);

/* Sizes that fix the workspace layout. */
typedef struct emrt_sizes {
    int64_t n_verts, n_tris, n_faces, n_objects; /* scene arrays */
    int32_t n_tx, n_rx;                          /* transmitters and receivers per frame */
} emrt_sizes;

/* Create / destroy a context.  Errors: EMRT_E_INVALID (NULL or out-of-range
 * config), EMRT_E_UNSUPPORTED (K > 5, n_freq > 4). */
int32_t emrt_ctx_create(const emrt_config* cfg, emrt_ctx** out);
int32_t emrt_ctx_destroy(emrt_ctx* ctx);

/* Bytes of device workspace for the given sizes (host call, no GPU work).
 * Errors: EMRT_E_INVALID (a size below 1), EMRT_E_UNSUPPORTED (n_tx > 4095,
 * n_rx >= 2^26, n_tris or n_verts >= 2^31, n_tx x rays_per_tx >= 2^32,
 * n_tx x n_rx + path_capacity >= 2^31). */
int32_t emrt_workspace_size(emrt_ctx* ctx, const emrt_sizes* sizes, size_t* bytes);
/* Bind a caller-allocated device workspace of at least emrt_workspace_size()
 * bytes (256-byte aligned).  The library carves all of its device state from
 * it; it stays owned by the caller and must outlive the context's work.
 * Errors: EMRT_E_WORKSPACE (too small / NULL), EMRT_E_INVALID (sizes). */
int32_t emrt_bind_workspace(emrt_ctx* ctx, void* device_ptr, size_t bytes);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): bind the
 * library's own static workspace of EMRT_STATIC_WORKSPACE_BYTES instead of a
 * caller buffer.  Same contract as emrt_bind_workspace otherwise (call
 * emrt_workspace_size first; the scene and everything after it must be set
 * again).  Allocates nothing: each GPU holds one such array from the first
 * bind on it until the process ends, and every context bound to it on that
 * GPU shares it, so only one may be in use at a time (a later bind takes it
 * over; overlapping use races).  Errors: EMRT_E_WORKSPACE (the sizes need
 * more than EMRT_STATIC_WORKSPACE_BYTES: the message gives both sizes),
 * EMRT_E_STATE (no sizes), EMRT_E_HIP (its device address). */
#define EMRT_STATIC_WORKSPACE_BYTES (64u << 20)
int32_t emrt_bind_static_workspace(emrt_ctx* ctx);
/* Stream for all subsequent work (a hipStream_t; NULL = default stream). */
int32_t emrt_set_stream(emrt_ctx* ctx, void* hip_stream);

/* Scene (Section IV: buildings and moving vehicles as triangle meshes, no
 * penetration).  A face is a set of coplanar triangles of one object and one
 * material, the unit of reflection and of path keys; triangles are wound
 * counter-clockwise seen from outside (used to find convex wedge edges).
 * Vertices of dynamic objects are in the object's local frame. */
typedef struct emrt_scene_desc {
    int64_t n_verts, n_tris, n_faces, n_objects;
    const float* verts;            /* device [n_verts][3] */
    const int32_t* tris;           /* device [n_tris][3] vertex indices */
    const int32_t* tri_face;       /* device [n_tris] face of each triangle */
    const int32_t* face_object;    /* device [n_faces] */
    const int32_t* face_material;  /* device [n_faces] */
    const uint8_t* object_dynamic; /* device [n_objects] 1 = moves with a per-frame transform */
    int32_t n_materials;           /* <= 256 */
    const double* material_eps;    /* host [n_materials][2] relative permittivity (re, im) */
} emrt_scene_desc;
/* Upload and preprocess a scene: index checks, face planes and triangle lists,
 * wedge edges, the trees over the static triangles and the static objects'
 * wedge edges (binned SAH, built once per scene).  Synchronises.  Errors: EMRT_E_INVALID
 * (sizes differ from the workspace's, index out of range, degenerate or
 * non-finite triangle), EMRT_E_STATE (no workspace). */
int32_t emrt_set_scene(emrt_ctx* ctx, const emrt_scene_desc* scene);
/* Replace the permittivity table without touching geometry (host array). */
int32_t emrt_set_materials(emrt_ctx* ctx, const double* material_eps, int32_t n_materials);
/* Constant reflection coefficients (Section IV, Table I, which describes its
 * wall and metal surfaces by a reflection coefficient alone: 0.8 and 0.9).
 * refl: host [n_materials], copied before the call returns.  0 keeps the
 * material's Fresnel coefficients from its permittivity (the state after
 * emrt_set_scene); g in (0, 1] gives it a coefficient of magnitude g at every
 * incidence angle for both polarisations, with a perfect conductor's signs
 * (TE -g, TM +g: the large-permittivity limit of the Fresnel forms), in
 * reflections and in the face terms of the diffraction coefficient.  Such a
 * material's permittivity gradient from emrt_backward is zero.
 * Errors: EMRT_E_INVALID (NULL, n_materials differs from the scene's, a value
 * outside [0, 1] or NaN), EMRT_E_STATE (no scene). */
int32_t emrt_set_reflection_coefficients(emrt_ctx* ctx, const double* refl, int32_t n_materials);

/* Per-frame state (Section III-A/C: moving objects and receivers; the base
 * station is static by default, but transmitter velocities are honoured).
 * All arrays are device pointers, copied into the workspace in stream order. */
typedef struct emrt_frame_desc {
    int64_t frame;
    double t_s;
    int32_t n_tx, n_rx;        /* must equal the workspace sizes */
    const double* obj_xform;   /* [n_dynamic][3][4] row-major rigid transforms, dynamic objects in id order */
    const double* obj_vel;     /* [n_dynamic][3] translational velocity */
    const double* tx_pos;      /* [n_tx][3] */
    const double* tx_vel;      /* [n_tx][3] */
    const double* tx_orient;   /* [n_tx][2] dipole (theta, phi), rad; ignored for ISO_V */
    const double* rx_pos;      /* [n_rx][3] */
    const double* rx_vel;      /* [n_rx][3] */
} emrt_frame_desc;
/* Errors: EMRT_E_INVALID (NULL, sizes differ, a null position or velocity
 * array, dynamic objects without transforms), EMRT_E_STATE (no scene). */
int32_t emrt_set_frame(emrt_ctx* ctx, const emrt_frame_desc* frame);

/* emrt_set_frame with every array of the descriptor a HOST pointer (layouts as
 * above; tx_orient may be NULL for zeros).  The arrays are packed into a
 * pinned buffer that the context owns and uploaded in one copy on its stream,
 * then scattered as in emrt_set_frame; they are read before the call returns,
 * so the caller may reuse them at once.  If the previous host upload is still
 * in flight the call first waits for it (the pinned buffer is single).  The
 * buffer is allocated on the first call and grown when the sizes grow; it is
 * freed by emrt_destroy.  Same errors as emrt_set_frame, plus EMRT_E_HIP when
 * the pinned buffer cannot be allocated. */
int32_t emrt_set_frame_host(emrt_ctx* ctx, const emrt_frame_desc* frame);

/* Run one frame.  discover = 1: launch rays from every transmitter, bounce
 * them, capture receivers and edges, merge the discovered keys with the cache
 * (Section II-A path caching); discover = 0: revalidate the cached keys only
 * (Section III-B).  Both then validate every key exactly plus line of sight
 * for every link, evaluate the fields and reduce per link; invalid keys are
 * dropped from the cache.  Errors: EMRT_E_STATE (no scene / frame). */
int32_t emrt_step(emrt_ctx* ctx, int32_t discover);

/* A discovery step whose rays start at receivers instead of transmitters
 * (Section II-A: rays traced backward from the receivers), for rediscovering
 * the links of a few receivers, e.g. those whose coherence statistics
 * triggered.  From each receiver rx_ids[i] (host [n_rx_ids], copied before the
 * call returns; 1..1024 entries, repeats allowed) rays_per_rx directions of
 * the same Fibonacci lattice are launched and bounced through the same trees
 * (K reflections); spheres of radius k_rx sqrt(4 pi / rays_per_rx) (L + s)
 * around the transmitters capture them after at least one reflection, and a
 * capture proposes the path from that transmitter to the receiver over the
 * faces in reverse order.  With diffraction on, an edge that a first segment
 * passes proposes the (tx, edge, rx) path for every transmitter.  The
 * proposals join the cache, and validation, fields and per-link sums run as
 * in emrt_step for every link, so other links are revalidated as on a cached
 * frame.  rx_ids x rays_per_rx may not exceed n_tx x rays_per_tx (the ray
 * buffers).  Errors: EMRT_E_STATE (no scene / frame, batched context),
 * EMRT_E_INVALID (count, rays or a receiver index out of range). */
int32_t emrt_step_rx(emrt_ctx* ctx, const int32_t* rx_ids, int32_t n_rx_ids, int32_t rays_per_rx);

/* Channel outputs of the last step.  Device buffers, any may be NULL.  Links
 * are ordered tx-major: link = tx * n_rx + rx.  Frequency-dependent arrays
 * are [n_freq][n_links]. */
typedef struct emrt_channel_view {
    double* H;        /* [n_freq][n_links][2] complex gain sum */
    double* P_coh;    /* [n_freq][n_links] P_tx |H|^2 */
    double* P_inc;    /* [n_freq][n_links] P_tx sum |a|^2 */
    double* tau_mean; /* [n_freq][n_links] power-weighted mean delay */
    double* tau_rms;  /* [n_freq][n_links] RMS delay spread */
    double* fd_mean;  /* [n_freq][n_links] mean Doppler shift (Section V-D) */
    double* fd_rms;   /* [n_freq][n_links] RMS Doppler spread (Section V-D) */
    int32_t* n_paths; /* [n_links] */
    uint32_t* flags;  /* [n_links] bit 0: line of sight present */
} emrt_channel_view;
int32_t emrt_read_channels(emrt_ctx* ctx, const emrt_channel_view* view);

/* Path lists of the last step, per link ordered by key (tx, rx, type, order,
 * ids).  Device buffers [n_links][cap][...], any may be NULL except count.
 * Returns EMRT_W_PATHS_TRUNCATED (after synchronising) when some link has
 * more than cap paths; the channel sums always use every path. */
typedef struct emrt_path_view {
    int32_t cap;
    int32_t* key;     /* [n_links][cap][9] tx, rx, type, order, id0..id4; type 0 line of sight, 1 specular
                         (ids: faces), 2 diffraction (id0: edge), 3 reflection then diffraction (face,
                         edge), 4 diffraction then reflection (edge, face) */
    int32_t* tri_ids; /* [n_links][cap][5] triangle of each reflection point (-1 at a diffraction) */
    double* a;        /* [n_links][cap][n_freq][2] complex gain */
    double* tau;      /* [n_links][cap] delay */
    double* fd;       /* [n_links][cap][n_freq] Doppler shift */
    float* angles;    /* [n_links][cap][4] departure az, el; arrival az, el (rad) */
    int32_t* count;   /* [n_links] paths written */
} emrt_path_view;
int32_t emrt_read_paths(emrt_ctx* ctx, const emrt_path_view* view);

/* Adjoint of the last step: gradients of a real loss L of the channels with
 * the path topology of that step held fixed (its valid paths are kept; their
 * interaction points and fields are rebuilt as functions of the parameters).
 * The paper computes channels only (received power, delay, Doppler:
 * Section III-C, Section V-D); gradients are an extension of it.
 *   dL_dH   device [n_freq][n_links][2]  dL/dRe H + j dL/dIm H, or NULL;
 *   dL_dP   device [n_freq][n_links]     dL/dP_coh, or NULL;
 * outputs (device, any may be NULL, overwritten):
 *   grad_eps        [n_materials][2]  dL/dRe eps + j dL/dIm eps;
 *   grad_tx_pos     [n_tx][3]         dL/d(transmitter position);
 *   grad_tx_orient  [n_tx][2]         dL/d(theta, phi) of the dipole (0 for EMRT_ANT_ISO_V).
 * Evaluated at the frame of the last step and the current materials.
 * Deterministic (fixed-order sums).  Errors: EMRT_E_STATE (no step, or
 * set_frame since the last step), EMRT_E_UNSUPPORTED (adjoint_materials is 0
 * or smaller than the scene's material count). */
int32_t emrt_backward(emrt_ctx* ctx, const double* dL_dH, const double* dL_dP, double* grad_eps, double* grad_tx_pos,
                      double* grad_tx_orient);

/* Coherence statistics over frames (Section III-B): every step updates, per
 * link and carrier, running sums of g = |H| and of its lagged products, and
 * per link the spatial-consistency triggers.  They tell the caller when to
 * rediscover (emrt_step with discover = 1) instead of revalidating the cache.
 * Readings (the paper prints the formulas, not their estimators):
 *   corr: Eq (1) as the normalised autocovariance of g at lags of 1..4
 *     frames, (mean_{t>=k} g_t g_{t-k} - m^2) / (mean g^2 - m^2), m = mean g,
 *     over the steps since the last reset (NaN while undefined);
 *   tc: Eq (2), sqrt(1/R^4 - 1) / (2 pi f_D theta^2), f_D = f_c |v_rx - v_tx| / c,
 *     theta the acute angle between the line of motion and the Tx -> Rx
 *     direction of the last step's frame (+inf when f_D theta^2 = 0);
 *   trigger: bit 0 the line of sight changed at the last step, bit 1 the set
 *     of first-order paths (one reflection or one diffraction) changed.
 * Device buffers, any may be NULL. */
#define EMRT_CORR_LAGS 4
typedef struct emrt_coherence_view {
    double* tc;        /* [n_freq][n_links] s */
    double* corr;      /* [n_freq][n_links][EMRT_CORR_LAGS] lags 1..4 frames */
    uint32_t* trigger; /* [n_links] */
} emrt_coherence_view;
/* R in (0, 1) (0.5 is a common choice); min_tc (host, may be NULL) gets the
 * smallest finite T_c over links and carriers (+inf if none), n_triggered
 * (host, may be NULL) the number of triggered links.  Synchronises.
 * Errors: EMRT_E_INVALID (R), EMRT_E_STATE (no step yet). */
int32_t emrt_read_coherence(emrt_ctx* ctx, double R, const emrt_coherence_view* view, double* min_tc,
                            int64_t* n_triggered);
/* Start the statistics afresh (a new trajectory segment). */
int32_t emrt_coherence_reset(emrt_ctx* ctx);

/* Batched stepping of several independent scenes (extension of the frame
 * step above to many cities at once).  A batch groups contexts that are
 * bound and have their scene set; it takes over their streams (all work goes
 * to the batch stream and up to n_streams - 1 helper streams of default
 * priority).  Per scene the step is the same as emrt_step; the bounces of
 * all scenes run as one persistent launch per bounce level, and the step is
 * captured once per (discover, cache parity) as a HIP graph and replayed.
 * Frames are set and results read through the member contexts
 * (emrt_set_frame, emrt_read_channels, ...); while batched, emrt_step on a
 * member returns EMRT_E_STATE.  emrt_batch_destroy gives every member back
 * the stream it had when the batch was created.  The batch workspace (device, caller-owned,
 * from emrt_batch_workspace_size) holds the per-level bounce arguments and
 * the chunk tables. */
typedef struct emrt_batch emrt_batch;
/* Errors: EMRT_E_STATE (a context unbound, without scene or already batched),
 * EMRT_E_INVALID (repeated context). */
int32_t emrt_batch_create(emrt_ctx* const* ctxs, int32_t n, emrt_batch** out);
int32_t emrt_batch_destroy(emrt_batch* batch);
int32_t emrt_batch_workspace_size(emrt_batch* batch, size_t* bytes);
int32_t emrt_batch_bind_workspace(emrt_batch* batch, void* device_ptr, size_t bytes);
/* hipStream_t of the batch (and of every member from now on). */
int32_t emrt_batch_set_stream(emrt_batch* batch, void* stream);
/* use_graph 0/1 (default 1), n_streams 1..16 (default 4), grid = workgroups
 * of the persistent multi-scene bounce launch (default 2048), chunk = rays a
 * wave takes per fetch from the launch's work counter: 32, 64 (default), 128,
 * 256, 512 or 1024 (EMRT_E_INVALID otherwise).  The primary rays' level
 * takes twice that (at most 1024), levels after the second at most 256. */
int32_t emrt_batch_set_options(emrt_batch* batch, int32_t use_graph, int32_t n_streams, int32_t grid, int32_t chunk);
/* Step every member (discover as in emrt_step).  Errors: EMRT_E_STATE (a
 * member without frame, or members at different cache parities),
 * EMRT_E_WORKSPACE, EMRT_E_HIP (graph capture or launch). */
int32_t emrt_batch_step(emrt_batch* batch, int32_t discover);
/* Choose grid, n_streams and chunk by timing real discovery steps of the
 * members' current frames: every combination of grid 1024..8192 (powers of
 * two), n_streams 1, 2, 4, 8 and chunk 64, 128, 256, 512, timed `repeats`
 * times (1..15) each after one warm-up step, the median compared (64 x
 * repeats + 1 steps; synchronises).  Any output pointer may be null. */
int32_t emrt_batch_autotune(emrt_batch* batch, int32_t repeats, int32_t* best_grid, int32_t* best_streams,
                            int32_t* best_chunk);
/* emrt_sync of every member; returns the most severe status. */
int32_t emrt_batch_sync(emrt_batch* batch);
int32_t emrt_batch_last_error(emrt_batch* batch, char* buf, size_t len);

/* Triangle hit per bounce of the last discovery step for launch directions
 * ray_ids (device [n]) of transmitter tx: out device [n][K+1], -1 miss,
 * -2 not traced (the ray ended earlier).  EMRT_E_STATE when the last
 * discovery step was a receiver-side one (emrt_step_rx). */
int32_t emrt_debug_ray_records(emrt_ctx* ctx, int32_t tx, const int32_t* ray_ids, int32_t n, int32_t* out);

/* Per-ray capture decisions (Section II-A: reception spheres of radius
 * k alpha (L + s) on the receivers; edge capture for diffraction), for
 * comparing them ray by ray.  emrt_debug_select_rays marks launch directions
 * ray_ids (device [n], each in [0, rays_per_tx)) of transmitter tx; n = 0
 * clears every mark.  The marks persist, and every later transmitter-side
 * discovery step logs each receiver and edge capture of a marked ray, up to
 * EMRT_CAPTURE_LOG_ROWS rows per step (EMRT_E_INVALID for a direction out of
 * range, EMRT_E_STATE before emrt_set_scene; batched steps log nothing).
 * emrt_debug_ray_captures copies the last discovery step's log into out
 * (device [cap][5] int32: tx, launch direction, bounce, kind (0 receiver,
 * 1 edge), receiver or edge id; in no particular order), sets *n_rows
 * (host) to the rows written and synchronises.  Returns
 * EMRT_W_PATHS_TRUNCATED when rows were dropped (the step logged more than
 * EMRT_CAPTURE_LOG_ROWS, or more than cap). */
#define EMRT_CAPTURE_LOG_ROWS (1 << 16)
int32_t emrt_debug_select_rays(emrt_ctx* ctx, int32_t tx, const int32_t* ray_ids, int32_t n);
int32_t emrt_debug_ray_captures(emrt_ctx* ctx, int32_t* out, int64_t cap, int64_t* n_rows);

/* Path cache (checkpoint / resume): the valid non-line-of-sight keys after
 * the last step, rows of 9 int32 as in emrt_path_view.key.  size and export
 * synchronise; import replaces the cache (device rows). */
int32_t emrt_cache_size(emrt_ctx* ctx, int64_t* n_keys);
int32_t emrt_cache_export(emrt_ctx* ctx, int32_t* keys, int64_t cap, int64_t* n_keys);
int32_t emrt_cache_import(emrt_ctx* ctx, const int32_t* keys, int64_t n_keys);

/* Counters of the last step (synchronises). */
typedef struct emrt_stats {
    int64_t rays_per_bounce[7]; /* live rays entering bounce b */
    int64_t n_candidates;       /* keys validated besides line of sight */
    int64_t n_valid;            /* valid paths including line of sight */
    int64_t n_cache;            /* cache size after the step */
    int64_t node_visits;        /* traversal counters (when stats are enabled) */
    int64_t tri_tests;
    int64_t segments;
    int64_t captures;
    int64_t n_static_tris, n_dynamic_tris, n_edges;
    uint32_t device_flags;
    double bounce_ms;           /* summed time of the bounce launches since timing was enabled */
    int32_t bounce_launches;
    double validate_ms;         /* summed time of the validation stage (construct, shadow, fields) */
    int32_t validate_launches;
    double static_tree_area;    /* static tree quality: summed surface area of every node below the
                                   root over the root's (the expected box tests of a random ray) */
    int64_t wide_box_tests;     /* child boxes tested in the static tree's 4-wide nodes (when stats are
                                   enabled); node_visits then counts the binary (dynamic tree) nodes */
    int64_t dyn_rebuilds;       /* builds of the moving objects' tree since the scene was set (steps
                                   outside a batch) */
    double dyn_tree_quality;    /* its quality at the last completed read-back (0: none yet) */
} emrt_stats;
int32_t emrt_read_stats(emrt_ctx* ctx, emrt_stats* out);
/* Optional instrumentation: stats = count traversal work (slower), timing =
 * HIP events around the bounce launches and the validation stage, summed over
 * the steps since this call (which resets the sums). */
int32_t emrt_set_instrumentation(emrt_ctx* ctx, int32_t stats, int32_t timing);

/* Wait for the context's stream; reports device-side flags of the work so
 * far: EMRT_W_CACHE_FULL (capacity reached) or EMRT_E_DEVICE_FLAG. */
int32_t emrt_sync(emrt_ctx* ctx);

const char* emrt_status_string(int32_t status);
/* Copy the last error message (NUL-terminated, truncated to len). */
int32_t emrt_last_error(emrt_ctx* ctx, char* buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* EMRT_H */
