/*
 * emrt_oracle.c -- plain FP64 CPU reference for the dynamic shooting-and-
 * bouncing-ray (SBR) EM path search and channel evaluation of
 * Wang & Manocha, "Dynamic EM Ray Tracing for Large Urban Scenes with
 * Multiple Receivers" (2023).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg load it.  It shares no code, header or table with the GPU
 * library, and the GPU library never calls it.
 *
 * Everything is brute force: every ray segment is tested against every
 * triangle, every receiver and every edge; there is no acceleration
 * structure.  Arithmetic is IEEE double without contraction (built with
 * -ffp-contract=off), except where the input contract fixes float32 values
 * (scene vertices, launch directions), which are promoted exactly.
 *
 * What the paper fixes and what is a reading:
 *   - Section II-A: the engine models direct, reflected and diffracted rays
 *     (scattering is out of scope), uses a BVH (here brute force, results are
 *     identical by construction) and caches propagation paths across frames.
 *   - Section III-B: valid paths are kept in a cache ("visibility hash table")
 *     and deleted once invalid.
 *   - Section III-C, Eq (3): LoS Doppler f_d = f_c (v/c) cos(theta); the base
 *     station is static by default.
 *   - Section IV: 50 dBm transmit power, ideal omnidirectional antennas, no
 *     penetration through walls.
 *   - Section V-D: mean Doppler shift and RMS Doppler spread per receiver.
 *   The paper gives no launch lattice, reception-sphere size, edge model,
 *   reflection-coefficient model or diffraction coefficient; those are
 *   readings, each stated at the function that implements it.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define ORC_C0 299792458.0

/* ------------------------------------------------------------------------ */
/* small FP64 vector helpers                                                 */
/* ------------------------------------------------------------------------ */
typedef struct { double x, y, z; } v3;

static v3 V(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 vadd(v3 a, v3 b) { return V(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 vsub(v3 a, v3 b) { return V(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 vmul(v3 a, double s) { return V(a.x * s, a.y * s, a.z * s); }
static double vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 vcross(v3 a, v3 b) {
    return V(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double vlen(v3 a) { return sqrt(vdot(a, a)); }
static v3 vnorm(v3 a) { double l = vlen(a); return vmul(a, 1.0 / l); }
static v3 ld3f(const float* p) { return V((double)p[0], (double)p[1], (double)p[2]); }
static v3 ld3d(const double* p) { return V(p[0], p[1], p[2]); }

/* vertex k (0..2) of triangle t from the expanded [T][9] float32 table */
static v3 tvert(const float* tv, int64_t t, int k) { return ld3f(tv + t * 9 + 3 * k); }

/* robustness margin (reading of "1e-4 rad from grazing or edge-hitting"):
 * distance margin 1e-4 * t + 1 mm at ray parameter t from the segment origin */
#define ROB_ANG 1.0e-4
#define ROB_FLOOR 1.0e-3
static double rob_m(double t) { return ROB_ANG * (t > 0 ? t : 0) + ROB_FLOOR; }

/* ------------------------------------------------------------------------ */
/* scene preprocessing                                                       */
/* ------------------------------------------------------------------------ */

/* World vertices of dynamic objects: each coordinate is
 * float32( ((R[i][0]*x + R[i][1]*y) + R[i][2]*z) + t[i] ) evaluated in double
 * with no fused multiply-add (reading: a fixed rounding rule so that every
 * implementation sees the identical float32 triangles).  vdyn[v] is the
 * dynamic-object rank owning vertex v, or -1 for static vertices, which are
 * copied unchanged.  xform is [O_d][3][4] row-major. */
void orc_world_verts(int32_t nv, const float* vloc, const int32_t* vdyn, const double* xform, float* vout) {
    for (int32_t v = 0; v < nv; v++) {
        int32_t o = vdyn[v];
        if (o < 0) {
            vout[3 * v + 0] = vloc[3 * v + 0];
            vout[3 * v + 1] = vloc[3 * v + 1];
            vout[3 * v + 2] = vloc[3 * v + 2];
            continue;
        }
        const double* m = xform + 12 * (int64_t)o;
        double x = vloc[3 * v], y = vloc[3 * v + 1], z = vloc[3 * v + 2];
        for (int i = 0; i < 3; i++) {
            double a = m[4 * i + 0] * x;
            double b = m[4 * i + 1] * y;
            double c = m[4 * i + 2] * z;
            double s = a + b;
            s = s + c;
            s = s + m[4 * i + 3];
            vout[3 * v + i] = (float)s;
        }
    }
}

/* Face plane (n, d) with n.x = d: the unit normal of the face's lowest-id
 * triangle, n = normalize((v1-v0) x (v2-v0)), d = n.v0.  A face is a set of
 * coplanar triangles of one object and one material; reflection happens at
 * faces (Section II-A's reflected rays; the face is the path-key unit). */
int32_t orc_face_planes(int32_t T, const float* tv, const int32_t* tri_face, int32_t F, double* plane) {
    int32_t* first = (int32_t*)malloc(sizeof(int32_t) * (size_t)F);
    for (int32_t f = 0; f < F; f++) first[f] = -1;
    for (int32_t t = 0; t < T; t++) {
        int32_t f = tri_face[t];
        if (f < 0 || f >= F) { free(first); return -1; }
        if (first[f] < 0) first[f] = t;
    }
    int32_t rc = 0;
    for (int32_t f = 0; f < F; f++) {
        if (first[f] < 0) { rc = -2; plane[4 * f] = plane[4 * f + 1] = plane[4 * f + 2] = plane[4 * f + 3] = 0; continue; }
        v3 a = tvert(tv, first[f], 0), b = tvert(tv, first[f], 1), c = tvert(tv, first[f], 2);
        v3 n = vcross(vsub(b, a), vsub(c, a));
        double l = vlen(n);
        if (!(l > 0)) { rc = -3; l = 1; }
        n = vmul(n, 1.0 / l);
        plane[4 * f + 0] = n.x;
        plane[4 * f + 1] = n.y;
        plane[4 * f + 2] = n.z;
        plane[4 * f + 3] = vdot(n, a);
    }
    free(first);
    return rc;
}

/* Wedge-edge extraction (reading; the paper names diffracted rays in
 * Section II-A but no edge model).  For every pair of non-parallel faces
 * (f < g) of one object: the triangle edges of f lying on plane g and the
 * triangle edges of g lying on plane f (both endpoints within 1 mm) both lie
 * on the planes' intersection line; their projected extents along
 * u = normalize(n_f x n_g) overlap in the wedge edge.  The wedge is kept when
 * it is convex seen from outside, with triangles wound counter-clockwise
 * seen from outside: the in-face direction of g, t_n, satisfies
 * t_n . n_f < 0.  The 0-face is f (the lower face id); the exterior angle is
 * n*pi with n = atan2(t_n.n_f, t_n.t_0) mapped to (0, 2pi) over pi.
 * Output rows: va, vb (vertex ids of the edge ends, va lower along u),
 * f0, fn, w0, wn (a vertex of each face off the edge line), sorted by (f0, fn).
 * Planes here are computed on the given (local) vertices. */
typedef struct { int32_t va, vb, f0, fn, w0, wn; double n; } orc_edge;

static int cmp_edge(const void* a, const void* b) {
    const orc_edge* x = (const orc_edge*)a;
    const orc_edge* y = (const orc_edge*)b;
    if (x->f0 != y->f0) return x->f0 < y->f0 ? -1 : 1;
    if (x->fn != y->fn) return x->fn < y->fn ? -1 : 1;
    return 0;
}

int32_t orc_edges(int32_t nv, const float* verts, int32_t T, const int32_t* tris, const int32_t* tri_face,
                  int32_t F, const int32_t* face_object, int32_t cap, int32_t* out, double* out_n) {
    (void)nv;
    /* planes from the local vertices */
    float* tv = (float*)malloc(sizeof(float) * 9 * (size_t)T);
    for (int32_t t = 0; t < T; t++)
        for (int k = 0; k < 3; k++)
            for (int c = 0; c < 3; c++) tv[9 * t + 3 * k + c] = verts[3 * tris[3 * t + k] + c];
    double* pl = (double*)malloc(sizeof(double) * 4 * (size_t)F);
    orc_face_planes(T, tv, tri_face, F, pl);
    /* triangles per face (CSR) and faces per object */
    int32_t* fcnt = (int32_t*)calloc((size_t)F + 1, sizeof(int32_t));
    for (int32_t t = 0; t < T; t++) fcnt[tri_face[t] + 1]++;
    for (int32_t f = 0; f < F; f++) fcnt[f + 1] += fcnt[f];
    int32_t* ftri = (int32_t*)malloc(sizeof(int32_t) * (size_t)T);
    int32_t* fill = (int32_t*)calloc((size_t)F, sizeof(int32_t));
    for (int32_t t = 0; t < T; t++) { int32_t f = tri_face[t]; ftri[fcnt[f] + fill[f]++] = t; }
    int32_t nobj = 0;
    for (int32_t f = 0; f < F; f++) if (face_object[f] + 1 > nobj) nobj = face_object[f] + 1;
    int32_t* ocnt = (int32_t*)calloc((size_t)nobj + 1, sizeof(int32_t));
    for (int32_t f = 0; f < F; f++) ocnt[face_object[f] + 1]++;
    for (int32_t o = 0; o < nobj; o++) ocnt[o + 1] += ocnt[o];
    int32_t* ofac = (int32_t*)malloc(sizeof(int32_t) * (size_t)F);
    int32_t* ofill = (int32_t*)calloc((size_t)nobj, sizeof(int32_t));
    for (int32_t f = 0; f < F; f++) { int32_t o = face_object[f]; ofac[ocnt[o] + ofill[o]++] = f; }

    orc_edge* E = (orc_edge*)malloc(sizeof(orc_edge) * (size_t)(cap > 0 ? cap : 1));
    int32_t ne = 0;
    const double tol = 1.0e-3;
    for (int32_t o = 0; o < nobj; o++) {
        for (int32_t ia = ocnt[o]; ia < ocnt[o + 1]; ia++) {
            for (int32_t ib = ocnt[o]; ib < ocnt[o + 1]; ib++) {
                int32_t f = ofac[ia], g = ofac[ib];
                if (!(f < g)) continue;
                v3 nf = ld3d(pl + 4 * f), ng = ld3d(pl + 4 * g);
                double df = pl[4 * f + 3], dg = pl[4 * g + 3];
                v3 u = vcross(nf, ng);
                if (vlen(u) < 1e-6) continue;
                u = vnorm(u);
                /* extents of f's edges on plane g, and g's edges on plane f */
                double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
                int32_t vlo[2] = {-1, -1}, vhi[2] = {-1, -1};
                for (int side = 0; side < 2; side++) {
                    int32_t ff = side ? g : f;
                    v3 on = side ? nf : ng;
                    double od = side ? df : dg;
                    for (int32_t q = fcnt[ff]; q < fcnt[ff + 1]; q++) {
                        int32_t t = ftri[q];
                        for (int k = 0; k < 3; k++) {
                            int32_t a = tris[3 * t + k], b = tris[3 * t + (k + 1) % 3];
                            v3 pa = ld3f(verts + 3 * a), pb = ld3f(verts + 3 * b);
                            if (fabs(vdot(on, pa) - od) > tol || fabs(vdot(on, pb) - od) > tol) continue;
                            if (vlen(vsub(pa, pb)) < tol) continue;
                            double sa = vdot(pa, u), sb = vdot(pb, u);
                            if (sa < lo[side] || (sa == lo[side] && a < vlo[side])) { lo[side] = sa; vlo[side] = a; }
                            if (sb < lo[side] || (sb == lo[side] && b < vlo[side])) { lo[side] = sb; vlo[side] = b; }
                            if (sa > hi[side] || (sa == hi[side] && a < vhi[side])) { hi[side] = sa; vhi[side] = a; }
                            if (sb > hi[side] || (sb == hi[side] && b < vhi[side])) { hi[side] = sb; vhi[side] = b; }
                        }
                    }
                }
                if (vlo[0] < 0 || vlo[1] < 0) continue;
                double a0 = lo[0] > lo[1] ? lo[0] : lo[1];
                double a1 = hi[0] < hi[1] ? hi[0] : hi[1];
                if (!(a1 - a0 > tol)) continue;
                int32_t va = lo[0] > lo[1] ? vlo[0] : (lo[1] > lo[0] ? vlo[1] : (vlo[0] < vlo[1] ? vlo[0] : vlo[1]));
                int32_t vb = hi[0] < hi[1] ? vhi[0] : (hi[1] < hi[0] ? vhi[1] : (vhi[0] < vhi[1] ? vhi[0] : vhi[1]));
                v3 P0 = ld3f(verts + 3 * va);
                /* off-line vertices of f and g: farthest from the edge line */
                int32_t w[2] = {-1, -1};
                for (int side = 0; side < 2; side++) {
                    int32_t ff = side ? g : f;
                    double best = -1;
                    for (int32_t q = fcnt[ff]; q < fcnt[ff + 1]; q++) {
                        int32_t t = ftri[q];
                        for (int k = 0; k < 3; k++) {
                            int32_t a = tris[3 * t + k];
                            v3 r = vsub(ld3f(verts + 3 * a), P0);
                            double dd = vlen(vsub(r, vmul(u, vdot(r, u))));
                            if (dd > best + 1e-12) { best = dd; w[side] = a; }
                        }
                    }
                }
                v3 r0 = vsub(ld3f(verts + 3 * w[0]), P0), rn = vsub(ld3f(verts + 3 * w[1]), P0);
                v3 t0 = vnorm(vsub(r0, vmul(u, vdot(r0, u))));
                v3 tn = vnorm(vsub(rn, vmul(u, vdot(rn, u))));
                double yy = vdot(tn, nf), xx = vdot(tn, t0);
                if (!(yy < -1e-9)) continue; /* not convex seen from outside */
                double phn = atan2(yy, xx);
                if (phn < 0) phn += 2 * M_PI;
                if (ne < cap) {
                    E[ne].va = va; E[ne].vb = vb; E[ne].f0 = f; E[ne].fn = g;
                    E[ne].w0 = w[0]; E[ne].wn = w[1]; E[ne].n = phn / M_PI;
                }
                ne++;
            }
        }
    }
    if (ne <= cap) {
        qsort(E, (size_t)ne, sizeof(orc_edge), cmp_edge);
        for (int32_t i = 0; i < ne; i++) {
            out[6 * i + 0] = E[i].va; out[6 * i + 1] = E[i].vb; out[6 * i + 2] = E[i].f0;
            out[6 * i + 3] = E[i].fn; out[6 * i + 4] = E[i].w0; out[6 * i + 5] = E[i].wn;
            out_n[i] = E[i].n;
        }
    }
    free(E); free(ofill); free(ofac); free(ocnt); free(fill); free(ftri); free(fcnt); free(pl); free(tv);
    return ne;
}

/* Launch direction i of N on a Fibonacci sphere (reading; the workloads only
 * say "Fibonacci sphere"): z = 1 - (2i+1)/N, r = sqrt(1 - z^2),
 * phi = i * pi * (3 - sqrt(5)), d = (r cos phi, r sin phi, z) in double,
 * then rounded to float32. */
void orc_fib_dirs(int32_t N, int32_t n, const int32_t* ids, float* out) {
    const double ga = M_PI * (3.0 - sqrt(5.0));
    for (int32_t k = 0; k < n; k++) {
        double i = (double)ids[k];
        double z = 1.0 - (2.0 * i + 1.0) / (double)N;
        double r = sqrt(1.0 - z * z);
        double ph = i * ga;
        out[3 * k + 0] = (float)(r * cos(ph));
        out[3 * k + 1] = (float)(r * sin(ph));
        out[3 * k + 2] = (float)z;
    }
}

/* ------------------------------------------------------------------------ */
/* geometric primitives                                                      */
/* ------------------------------------------------------------------------ */

/* Moller-Trumbore line/triangle in double, two-sided, edges inclusive.
 * Returns 1 and the line parameter t (any sign) when o + t d meets the
 * triangle; 0 when it misses or lies in the triangle's plane. */
static int line_tri_t(v3 o, v3 d, v3 a, v3 b, v3 c, double* t_out) {
    v3 e1 = vsub(b, a), e2 = vsub(c, a);
    v3 p = vcross(d, e2);
    double det = vdot(e1, p);
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    v3 s = vsub(o, a);
    double u = vdot(s, p) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    v3 q = vcross(s, e1);
    double v = vdot(d, q) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    *t_out = vdot(e2, q) * inv;
    return 1;
}

/* The ray o + t d, t > 0, meets the triangle: returns 1 and t. */
static int tri_hit(v3 o, v3 d, v3 a, v3 b, v3 c, double* t_out) {
    double t;
    if (!line_tri_t(o, d, a, b, c, &t) || !(t > 0.0)) return 0;
    *t_out = t;
    return 1;
}

/* distance from point p to segment [a, b] */
static double pt_seg_dist(v3 p, v3 a, v3 b) {
    v3 ab = vsub(b, a);
    double l2 = vdot(ab, ab);
    double s = l2 > 0 ? vdot(vsub(p, a), ab) / l2 : 0.0;
    if (s < 0) s = 0;
    if (s > 1) s = 1;
    return vlen(vsub(p, vadd(a, vmul(ab, s))));
}

/* Closest points between segment P(s) = p0 + s*(p1-p0), s in [0,1], and
 * Q(u) = q0 + u*(q1-q0), u in [0,1]; returns the distance and the
 * parameters.  Classic clamped normal-equation solution. */
static double seg_seg(v3 p0, v3 p1, v3 q0, v3 q1, double* s_out, double* u_out) {
    v3 d1 = vsub(p1, p0), d2 = vsub(q1, q0), r = vsub(p0, q0);
    double a = vdot(d1, d1), e = vdot(d2, d2), f = vdot(d2, r);
    double s, u;
    if (a <= 0 && e <= 0) { s = u = 0; }
    else if (a <= 0) { s = 0; u = f / e; u = u < 0 ? 0 : (u > 1 ? 1 : u); }
    else {
        double c = vdot(d1, r);
        if (e <= 0) { u = 0; s = -c / a; s = s < 0 ? 0 : (s > 1 ? 1 : s); }
        else {
            double b = vdot(d1, d2), den = a * e - b * b;
            s = den > 0 ? (b * f - c * e) / den : 0.0;
            s = s < 0 ? 0 : (s > 1 ? 1 : s);
            u = (b * s + f) / e;
            if (u < 0) { u = 0; s = -c / a; s = s < 0 ? 0 : (s > 1 ? 1 : s); }
            else if (u > 1) { u = 1; s = (b - c) / a; s = s < 0 ? 0 : (s > 1 ? 1 : s); }
        }
    }
    *s_out = s; *u_out = u;
    return vlen(vsub(vadd(p0, vmul(d1, s)), vadd(q0, vmul(d2, u))));
}

/* segment vs axis-aligned box inflated by m (slab test) */
static int seg_box(v3 o, v3 d, double t1, const double* lo, const double* hi) {
    double t0 = 0.0, tt1 = t1;
    double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    for (int k = 0; k < 3; k++) {
        if (dd[k] == 0.0) { if (oo[k] < lo[k] || oo[k] > hi[k]) return 0; continue; }
        double a = (lo[k] - oo[k]) / dd[k], b = (hi[k] - oo[k]) / dd[k];
        if (a > b) { double tmp = a; a = b; b = tmp; }
        if (a > t0) t0 = a;
        if (b < tt1) tt1 = b;
        if (t0 > tt1) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* shooting and bouncing rays                                                */
/* ------------------------------------------------------------------------ */

/* Bounce loop for one transmitter and a subset of its N launch directions
 * (reading of Section II-A's reflected/diffracted rays as SBR shooting from
 * the transmitter):
 *   for b = 0..K: closest hit over all triangles, two-sided, t > 0, the
 *   previous face excluded, ties broken by the smallest (t, tri id);
 *   receiver capture on segment b >= 1: receiver r is captured when
 *   s = (r-o).d lies in (0, t_end) and its distance to the ray is below
 *   k_rx * alpha * (L_acc + s), alpha = sqrt(4 pi / N) (reception sphere);
 *   edge capture on segment 0 (diffraction >= 1), and on segment 1 as well
 *   (diffraction = 2: reflection then diffraction): the ray passes within
 *   k_rx * alpha * (L_acc + s) of an edge's interior before t_end;
 *   reflect: d' = d - 2 (d.n) n about the face plane, L_acc += t;
 *   stop on a miss or after K reflections (no power threshold).
 * Direct-segment (b = 0) receiver captures are not emitted: line of sight is
 * tested deterministically for every link.
 * Outputs per ray: hit_tri[K+1] (triangle id, -1 miss, -2 not traced) and,
 * when want_robust, robust = 1 iff every segment keeps the distance margin
 * rob_m from every decision (grazing, triangle edges, near-coincident hits,
 * capture thresholds).  Capture rows (ray index, b, rx) and edge rows
 * (ray index, edge, b) are appended; counts beyond capacity are still
 * counted. */
int32_t orc_trace(int32_t T, const float* tv, const int32_t* tri_face, const double* plane,
                  const double* tx, int32_t N, int32_t n_rays, const int32_t* ray_ids, int32_t K,
                  int32_t n_rx, const double* rx, double k_rx, int32_t n_edges, const double* edge_p,
                  int32_t diffraction, int32_t want_robust, const double* sphere,
                  int32_t* hit_tri, uint8_t* robust, int64_t cap_cap, int32_t* cap_out, int64_t* n_cap,
                  int64_t edge_cap, int32_t* edge_out, int64_t* n_edge_out) {
    const double alpha = sqrt(4.0 * M_PI / (double)N);
    const double sin_graze = sin(ROB_ANG);
    float* dirs = (float*)malloc(sizeof(float) * 3 * (size_t)(n_rays > 0 ? n_rays : 1));
    orc_fib_dirs(N, n_rays, ray_ids, dirs);
    /* triangle boxes for the robustness pre-filter */
    double* tbox = NULL;
    if (want_robust) {
        tbox = (double*)malloc(sizeof(double) * 6 * (size_t)(T > 0 ? T : 1));
        for (int32_t t = 0; t < T; t++) {
            for (int c = 0; c < 3; c++) {
                double a = tv[9 * t + c], b = tv[9 * t + 3 + c], d = tv[9 * t + 6 + c];
                tbox[6 * t + c] = fmin(a, fmin(b, d));
                tbox[6 * t + 3 + c] = fmax(a, fmax(b, d));
            }
        }
    }
    v3 sc = V(sphere[0], sphere[1], sphere[2]);
    double sr = sphere[3];
    int64_t ncap = 0, nedge = 0;

#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t k = 0; k < n_rays; k++) {
        v3 o = ld3d(tx);
        v3 d = vnorm(ld3f(dirs + 3 * k));
        double L = 0.0;
        int32_t prev_face = -1;
        int rob = 1;
        for (int b = 0; b <= K; b++) hit_tri[(int64_t)k * (K + 1) + b] = -2;
        for (int b = 0; b <= K; b++) {
            double best_t = INFINITY;
            int32_t best = -1;
            for (int32_t t = 0; t < T; t++) {
                if (tri_face[t] == prev_face) continue;
                double th;
                if (tri_hit(o, d, tvert(tv, t, 0), tvert(tv, t, 1), tvert(tv, t, 2), &th)) {
                    if (th < best_t || (th == best_t && t < best)) { best_t = th; best = t; }
                }
            }
            hit_tri[(int64_t)k * (K + 1) + b] = best;
            int hit = best >= 0;
            double t_end = hit ? best_t : INFINITY;
            /* segment end used by the robustness checks on a miss: exit from
             * the scene's bounding sphere */
            double t_chk = t_end;
            if (!hit) {
                v3 oc = vsub(o, sc);
                double bb = vdot(oc, d), cc = vdot(oc, oc) - sr * sr;
                double disc = bb * bb - cc;
                t_chk = disc > 0 ? -bb + sqrt(disc) : 0.0;
                if (t_chk < 0) t_chk = 0;
            }
            if (want_robust && rob) {
                if (hit) {
                    int32_t f = tri_face[best];
                    v3 n = ld3d(plane + 4 * f);
                    if (fabs(vdot(d, n)) < sin_graze) rob = 0;                          /* R1 grazing */
                    v3 p = vadd(o, vmul(d, best_t));
                    double m = rob_m(best_t);
                    for (int e = 0; e < 3 && rob; e++)                                   /* R2 near own edges */
                        if (pt_seg_dist(p, tvert(tv, best, e), tvert(tv, best, (e + 1) % 3)) < m) rob = 0;
                }
                double mmax = rob_m(t_chk);
                v3 p1 = vadd(o, vmul(d, t_chk));
                for (int32_t t = 0; t < T && rob; t++) {
                    double lo[3] = {tbox[6 * t] - mmax, tbox[6 * t + 1] - mmax, tbox[6 * t + 2] - mmax};
                    double hi[3] = {tbox[6 * t + 3] + mmax, tbox[6 * t + 4] + mmax, tbox[6 * t + 5] + mmax};
                    if (!seg_box(o, d, t_chk + mmax, lo, hi)) continue;
                    for (int e = 0; e < 3; e++) {                                         /* R3 near-miss edges */
                        double s, u;
                        double dist = seg_seg(o, p1, tvert(tv, t, e), tvert(tv, t, (e + 1) % 3), &s, &u);
                        if (dist < rob_m(s * t_chk)) { rob = 0; break; }
                    }
                    if (!rob) break;
                    if (hit && t != best && tri_face[t] != prev_face) {                   /* R4 near-coincident hit */
                        double th;
                        if (tri_hit(o, d, tvert(tv, t, 0), tvert(tv, t, 1), tvert(tv, t, 2), &th) &&
                            fabs(th - best_t) < rob_m(best_t) && tri_face[t] != tri_face[best])
                            rob = 0;
                    }
                }
            }
            /* receiver capture (segments after at least one reflection) */
            if (b >= 1) {
                for (int32_t r = 0; r < n_rx; r++) {
                    v3 w = vsub(ld3d(rx + 3 * r), o);
                    double s = vdot(w, d);
                    double rho2 = vdot(w, w) - s * s;
                    double rho = rho2 > 0 ? sqrt(rho2) : 0.0;
                    double rs = k_rx * alpha * (L + s);
                    if (want_robust && rob) {                                             /* R5 capture margins */
                        double m = rob_m(s);
                        if (s > -m && s < t_chk + m) {
                            if (fabs(rho - rs) < m) rob = 0;
                            if (rho < rs + m && (fabs(s) < m || (hit && fabs(s - t_end) < m))) rob = 0;
                        }
                    }
                    if (s > 0.0 && s < t_end && rho < rs) {
                        int64_t slot;
#pragma omp atomic capture
                        slot = ncap++;
                        if (slot < cap_cap) {
                            cap_out[3 * slot + 0] = k;
                            cap_out[3 * slot + 1] = b;
                            cap_out[3 * slot + 2] = r;
                        }
                    }
                }
            }
            /* edge capture on the first segment, and with diffraction = 2 on
             * the second (after one reflection) too; radius k_rx alpha (L + s) */
            if ((b == 0 && diffraction) || (b == 1 && diffraction == 2)) {
                for (int32_t e = 0; e < n_edges; e++) {
                    v3 q0 = ld3d(edge_p + 6 * e), q1 = ld3d(edge_p + 6 * e + 3);
                    v3 ev = vsub(q1, q0);
                    v3 w0 = vsub(o, q0);
                    double a = vdot(d, d), bb = vdot(d, ev), c = vdot(ev, ev);
                    double dd = vdot(d, w0), ee = vdot(ev, w0);
                    double den = a * c - bb * bb;
                    if (!(den > 1e-12 * a * c)) continue;
                    double s = (bb * ee - c * dd) / den;
                    double u = (a * ee - bb * dd) / den;
                    double dist = vlen(vsub(vadd(o, vmul(d, s)), vadd(q0, vmul(ev, u))));
                    double re = k_rx * alpha * (L + s);
                    double elen = sqrt(c);
                    if (want_robust && rob) {
                        double m = rob_m(s);
                        if (dist < re + m && s > -m && s < t_chk + m && u * elen > -m && (1 - u) * elen > -m) {
                            if (fabs(dist - re) < m || fabs(s) < m || (hit && fabs(s - t_end) < m) ||
                                fabs(u * elen) < m || fabs((1 - u) * elen) < m)
                                rob = 0;
                        }
                    }
                    if (s > 0.0 && s < t_end && u > 0.0 && u < 1.0 && dist < re) {
                        int64_t slot;
#pragma omp atomic capture
                        slot = nedge++;
                        if (slot < edge_cap) {
                            edge_out[3 * slot + 0] = k;
                            edge_out[3 * slot + 1] = e;
                            edge_out[3 * slot + 2] = b;
                        }
                    }
                }
            }
            if (!hit || b == K) break;
            int32_t f = tri_face[best];
            v3 n = ld3d(plane + 4 * f);
            o = vadd(o, vmul(d, best_t));
            d = vsub(d, vmul(n, 2.0 * vdot(d, n)));
            L += best_t;
            prev_face = f;
        }
        if (robust) robust[k] = (uint8_t)(want_robust ? rob : 0);
    }
    *n_cap = ncap;
    *n_edge_out = nedge;
    free(dirs);
    free(tbox);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* exact path construction and validation                                    */
/* ------------------------------------------------------------------------ */

/* point-in-triangle for a point on (or numerically next to) the triangle's
 * plane: signed areas after dropping the dominant normal axis; edges count as
 * inside.  Returns the distance to the nearest triangle edge through *edist. */
static int in_tri(v3 p, v3 a, v3 b, v3 c, double* edist) {
    v3 n = vcross(vsub(b, a), vsub(c, a));
    double ax = fabs(n.x), ay = fabs(n.y), az = fabs(n.z);
    double P[2], A[2], B[2], C[2];
    if (az >= ax && az >= ay) { P[0] = p.x; P[1] = p.y; A[0] = a.x; A[1] = a.y; B[0] = b.x; B[1] = b.y; C[0] = c.x; C[1] = c.y; }
    else if (ay >= ax) { P[0] = p.z; P[1] = p.x; A[0] = a.z; A[1] = a.x; B[0] = b.z; B[1] = b.x; C[0] = c.z; C[1] = c.x; }
    else { P[0] = p.y; P[1] = p.z; A[0] = a.y; A[1] = a.z; B[0] = b.y; B[1] = b.z; C[0] = c.y; C[1] = c.z; }
    double w0 = (B[0] - P[0]) * (C[1] - P[1]) - (B[1] - P[1]) * (C[0] - P[0]);
    double w1 = (C[0] - P[0]) * (A[1] - P[1]) - (C[1] - P[1]) * (A[0] - P[0]);
    double w2 = (A[0] - P[0]) * (B[1] - P[1]) - (A[1] - P[1]) * (B[0] - P[0]);
    int inside = (w0 >= 0 && w1 >= 0 && w2 >= 0) || (w0 <= 0 && w1 <= 0 && w2 <= 0);
    if (edist) {
        double m = pt_seg_dist(p, a, b);
        double m2 = pt_seg_dist(p, b, c), m3 = pt_seg_dist(p, c, a);
        if (m2 < m) m = m2;
        if (m3 < m) m = m3;
        *edist = m;
    }
    return inside;
}

/* Occlusion of the open segment p0 -> p1 (parameter in (0, 1)) by any
 * triangle outside the excluded faces (Section IV: opaque geometry, no
 * penetration).  Sets *amb when the decision is within the margin
 * m = 1 mm + 1e-6 * |p1 - p0| and could flip under float32 geometry: a
 * triangle's edge passes within m of the segment, or a triangle meets the
 * segment's line within m of an end point (a face coplanar with the face of
 * an interaction point and overlapping it there, such as the roofs of two
 * overlapping vehicles: whether it blocks is a matter of rounding). */
static int occluded3(int32_t T, const float* tv, const int32_t* tri_face, v3 p0, v3 p1, int32_t xa, int32_t xb,
                     int32_t xc, int* amb) {
    v3 d = vsub(p1, p0);
    double len = vlen(d);
    double m = 1.0e-3 + 1.0e-6 * len;
    int occ = 0;
    for (int32_t t = 0; t < T; t++) {
        int32_t f = tri_face[t];
        if (f == xa || f == xb || f == xc) continue;
        v3 a = tvert(tv, t, 0), b = tvert(tv, t, 1), c = tvert(tv, t, 2);
        double th;
        if (line_tri_t(p0, d, a, b, c, &th)) {
            if (th > 0.0 && th < 1.0) occ = 1;
            if (amb && (fabs(th) * len < m || fabs(1.0 - th) * len < m)) *amb = 1;
        }
        if (amb && !*amb) {
            double lo[3], hi[3];
            lo[0] = fmin(a.x, fmin(b.x, c.x)) - m; hi[0] = fmax(a.x, fmax(b.x, c.x)) + m;
            lo[1] = fmin(a.y, fmin(b.y, c.y)) - m; hi[1] = fmax(a.y, fmax(b.y, c.y)) + m;
            lo[2] = fmin(a.z, fmin(b.z, c.z)) - m; hi[2] = fmax(a.z, fmax(b.z, c.z)) + m;
            if (seg_box(p0, d, 1.0, lo, hi)) {
                v3 vv[3] = {a, b, c};
                for (int e = 0; e < 3; e++) {
                    double s, u;
                    if (seg_seg(p0, p1, vv[e], vv[(e + 1) % 3], &s, &u) < m) { *amb = 1; break; }
                }
            }
        }
        if (occ && !amb) return 1;
    }
    return occ;
}

static int occluded(int32_t T, const float* tv, const int32_t* tri_face, v3 p0, v3 p1, int32_t xa, int32_t xb, int* amb) {
    return occluded3(T, tv, tri_face, p0, p1, xa, xb, -1, amb);
}

/* mirror point p about plane (n, dd) */
static v3 mirror(v3 p, v3 n, double dd) { return vsub(p, vmul(n, 2.0 * (vdot(n, p) - dd))); }

/* Edge frame at the current vertices: P0, P1, unit e, in-face direction t0
 * of the 0-face and its outward normal n0 (pointing away from the n-face). */
typedef struct { v3 P0, P1, e, t0, n0; double len, n; int32_t f0, fn; } orc_wedge;

static orc_wedge wedge_at(const float* verts, const int32_t* erow, double wn) {
    orc_wedge w;
    w.P0 = ld3f(verts + 3 * erow[0]);
    w.P1 = ld3f(verts + 3 * erow[1]);
    v3 ev = vsub(w.P1, w.P0);
    w.len = vlen(ev);
    w.e = vmul(ev, 1.0 / w.len);
    v3 r0 = vsub(ld3f(verts + 3 * erow[4]), w.P0);
    v3 rn = vsub(ld3f(verts + 3 * erow[5]), w.P0);
    w.t0 = vnorm(vsub(r0, vmul(w.e, vdot(r0, w.e))));
    v3 tn = vnorm(vsub(rn, vmul(w.e, vdot(rn, w.e))));
    v3 n0 = vcross(w.e, w.t0);
    if (vdot(n0, tn) > 0) n0 = vmul(n0, -1.0);
    w.n0 = n0;
    w.n = wn;
    w.f0 = erow[2];
    w.fn = erow[3];
    return w;
}

/* angle of point p about the wedge, measured from the 0-face through the
 * exterior, in [0, 2pi) */
static double wedge_angle(const orc_wedge* w, v3 p) {
    v3 v = vsub(p, w->P0);
    double ph = atan2(vdot(v, w->n0), vdot(v, w->t0));
    if (ph < 0) ph += 2 * M_PI;
    return ph;
}

/* Range check of one key row [tx, rx, type, order, id0..id4] before any
 * array is indexed with it: tx in [0, n_tx), rx in [0, n_rx); type 0 (line of
 * sight) has order 0; type 1 (specular) order 1..5 with that many face ids in
 * [0, F); type 2 (diffraction) order 1 with an edge id in [0, E); types 3 and
 * 4 (one reflection and one diffraction) order 2 with (face, edge) or (edge,
 * face).  A malformed key (from the code under test) is reported as such and
 * never read further, so it fails a comparison instead of corrupting the
 * oracle's own state. */
static int key_ok(const int32_t* k, int32_t n_tx, int32_t n_rx, int32_t F, int32_t E) {
    if (k[0] < 0 || k[0] >= n_tx || k[1] < 0 || k[1] >= n_rx) return 0;
    const int32_t type = k[2], order = k[3];
    switch (type) {
        case 0: return order == 0;
        case 1:
            if (order < 1 || order > 5) return 0;
            for (int i = 0; i < order; i++)
                if (k[4 + i] < 0 || k[4 + i] >= F) return 0;
            return 1;
        case 2: return order == 1 && k[4] >= 0 && k[4] < E;
        case 3: return order == 2 && k[4] >= 0 && k[4] < F && k[5] >= 0 && k[5] < E;
        case 4: return order == 2 && k[4] >= 0 && k[4] < E && k[5] >= 0 && k[5] < F;
        default: return 0;
    }
}

/* Number of malformed rows among n_keys keys; bad[q] = 1 for each (bad may
 * be NULL). */
int32_t orc_check_keys(int32_t n_keys, const int32_t* keys, int32_t n_tx, int32_t n_rx, int32_t F, int32_t E,
                       uint8_t* bad) {
    int32_t nb = 0;
    for (int32_t q = 0; q < n_keys; q++) {
        const int ok = key_ok(keys + 9 * q, n_tx, n_rx, F, E);
        if (bad) bad[q] = (uint8_t)!ok;
        nb += !ok;
    }
    return nb;
}

/* Validation of path keys (Section II-A's direct, reflected and diffracted
 * rays; Section III-B's cache revalidation).  keys rows are
 * [tx, rx, type, order, id0..id4] with type 0 = line of sight, 1 = specular
 * (ids = face sequence), 2 = first-order edge diffraction (id0 = edge).
 *   Specular (image method): s_0 = Tx, s_k = mirror(s_{k-1}, plane f_k);
 *   back-track from Rx: x_k = segment(x_{k+1} -> s_k) meets plane f_k at a
 *   parameter in (0, 1); every x_k lies in a triangle of f_k (reported id:
 *   lowest containing triangle); every leg is unoccluded by triangles
 *   outside the faces of its two ends.
 *   Diffraction: Keller point Q on the edge line (equal angles with the
 *   edge: unfold Rx about the edge), strictly inside the edge; Tx and Rx in
 *   the exterior wedge (0 < phi', phi < n pi); |Q - Rx| <= diff_max_leg;
 *   both legs unoccluded outside the two wedge faces.
 *   Reflection then diffraction (type 3, ids = face, edge) and diffraction
 *   then reflection (type 4, ids = edge, face), order 2: the diffraction
 *   rules applied to the image of Tx (type 3) or of Rx (type 4) in the face
 *   plane; the reflection point where the segment from Q to that image
 *   crosses the plane (parameter in (0, 1), inside the face, which is not a
 *   wedge face); the receiver-side length |Q - image| or |Q - Rx| within
 *   diff_max_leg; three legs unoccluded outside the faces of their ends.
 * ambiguous = 1 when a decision is within its margin (containment within
 * 1e-6 m of a triangle edge, an image parameter within 1e-9 of its ends, a
 * shadow leg within 1 mm + 1e-6 |leg| of a triangle edge, a Keller point
 * within rob_m of an edge end, phi within 1e-4 rad of a face). */
int32_t orc_validate(int32_t T, const float* tv, const int32_t* tri_face, const double* plane, int32_t F,
                     int32_t E, int32_t n_tx, int32_t n_rx, const int32_t* face_off, const int32_t* face_tris,
                     const float* verts, const int32_t* edges, const double* edge_n, const double* txp,
                     const double* rxp, double diff_max_leg, int32_t n_keys, const int32_t* keys, uint8_t* valid,
                     uint8_t* ambiguous, int32_t* tri_ids, double* points) {
    int32_t n_bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : n_bad)
    for (int32_t q = 0; q < n_keys; q++) {
        const int32_t* key = keys + 9 * q;
        for (int i = 0; i < 5; i++) tri_ids[5 * q + i] = -1;
        for (int i = 0; i < 15; i++) points[15 * q + i] = 0.0;
        if (!key_ok(key, n_tx, n_rx, F, E)) {  /* malformed: invalid, never indexed */
            valid[q] = 0;
            ambiguous[q] = 0;
            n_bad++;
            continue;
        }
        v3 s = ld3d(txp + 3 * key[0]);
        v3 r = ld3d(rxp + 3 * key[1]);
        int type = key[2], order = key[3];
        int ok = 1, amb = 0;
        if (type == 0) {
            if (occluded(T, tv, tri_face, s, r, -1, -1, &amb)) ok = 0;
        } else if (type == 1) {
            v3 img[6];  /* Tx and its images through up to 5 faces */
            v3 x[7];    /* Tx, up to 5 reflection points, Rx */
            img[0] = s;
            for (int i = 1; i <= order; i++) {
                int32_t f = key[3 + i];
                img[i] = mirror(img[i - 1], ld3d(plane + 4 * f), plane[4 * f + 3]);
            }
            v3 cur = r;
            for (int i = order; i >= 1 && ok; i--) {
                int32_t f = key[3 + i];
                v3 n = ld3d(plane + 4 * f);
                v3 dv = vsub(img[i], cur);
                double den = vdot(n, dv);
                if (den == 0.0) { ok = 0; break; }
                double tt = (plane[4 * f + 3] - vdot(n, cur)) / den;
                if (!(tt > 0.0 && tt < 1.0)) { ok = 0; break; }
                if (tt < 1e-9 || tt > 1 - 1e-9) amb = 1;
                x[i] = vadd(cur, vmul(dv, tt));
                cur = x[i];
                int32_t found = -1;
                double ed = 0;
                for (int32_t j = face_off[f]; j < face_off[f + 1]; j++) {
                    int32_t t = face_tris[j];
                    double e1;
                    if (in_tri(x[i], tvert(tv, t, 0), tvert(tv, t, 1), tvert(tv, t, 2), &e1)) {
                        if (found < 0 || t < found) { found = t; ed = e1; }
                    }
                }
                if (found < 0) { ok = 0; break; }
                if (ed < 1e-6) amb = 1;
                tri_ids[5 * q + i - 1] = found;
                points[15 * q + 3 * (i - 1) + 0] = x[i].x;
                points[15 * q + 3 * (i - 1) + 1] = x[i].y;
                points[15 * q + 3 * (i - 1) + 2] = x[i].z;
            }
            if (ok) {
                x[0] = s;
                x[order + 1] = r;
                for (int i = 0; i <= order && ok; i++) {
                    int32_t xa = i >= 1 ? key[3 + i] : -1;
                    int32_t xb = i + 1 <= order ? key[4 + i] : -1;
                    if (occluded(T, tv, tri_face, x[i], x[i + 1], xa, xb, &amb)) ok = 0;
                }
            }
        } else if (type == 2) {
            int32_t e = key[4];
            orc_wedge w = wedge_at(verts, edges + 6 * e, edge_n[e]);
            double zs = vdot(vsub(s, w.P0), w.e), zr = vdot(vsub(r, w.P0), w.e);
            double rs = vlen(vsub(vsub(s, w.P0), vmul(w.e, zs)));
            double rr = vlen(vsub(vsub(r, w.P0), vmul(w.e, zr)));
            if (!(rs + rr > 0)) ok = 0;
            double zq = ok ? zs + (zr - zs) * rs / (rs + rr) : 0.0;
            if (ok && !(zq > 0.0 && zq < w.len)) ok = 0;
            v3 Q = vadd(w.P0, vmul(w.e, zq));
            if (ok) {
                double m = rob_m(vlen(vsub(Q, s)));
                if (zq < m || w.len - zq < m) amb = 1;
                double php = wedge_angle(&w, s), ph = wedge_angle(&w, r);
                if (!(php > 0 && php < w.n * M_PI && ph > 0 && ph < w.n * M_PI)) ok = 0;
                if (php < 1e-4 || fabs(php - w.n * M_PI) < 1e-4 || ph < 1e-4 || fabs(ph - w.n * M_PI) < 1e-4) amb = 1;
            }
            if (ok && !(vlen(vsub(Q, r)) <= diff_max_leg)) ok = 0;
            if (ok) {
                points[15 * q + 0] = Q.x;
                points[15 * q + 1] = Q.y;
                points[15 * q + 2] = Q.z;
                if (occluded(T, tv, tri_face, s, Q, w.f0, w.fn, &amb)) ok = 0;
                else if (occluded(T, tv, tri_face, Q, r, w.f0, w.fn, &amb)) ok = 0;
            }
        } else if (type == 3 || type == 4) {
            /* one reflection and one diffraction: the reflection is unfolded by
             * the image of the transmitter (3, reflection first) or of the
             * receiver (4, diffraction first) in the face plane; the Keller
             * point joins the real end to that image, and the reflection point
             * is where the segment from the Keller point to the image crosses
             * the plane. */
            const int rd = type == 3;
            int32_t f = rd ? key[4] : key[5], e = rd ? key[5] : key[4];
            orc_wedge w = wedge_at(verts, edges + 6 * e, edge_n[e]);
            v3 n = ld3d(plane + 4 * f);
            double dpl = plane[4 * f + 3];
            v3 a = rd ? mirror(s, n, dpl) : s;  /* source side of the edge (unfolded) */
            v3 b = rd ? r : mirror(r, n, dpl);  /* receiver side (unfolded) */
            if (f == w.f0 || f == w.fn || order != 2) ok = 0;
            double za = vdot(vsub(a, w.P0), w.e), zb = vdot(vsub(b, w.P0), w.e);
            double ra = vlen(vsub(vsub(a, w.P0), vmul(w.e, za)));
            double rb = vlen(vsub(vsub(b, w.P0), vmul(w.e, zb)));
            if (ok && !(ra + rb > 0)) ok = 0;
            double zq = ok ? za + (zb - za) * ra / (ra + rb) : 0.0;
            if (ok && !(zq > 0.0 && zq < w.len)) ok = 0;
            v3 Q = vadd(w.P0, vmul(w.e, zq));
            if (ok) {
                double m = rob_m(vlen(vsub(Q, a)));
                if (zq < m || w.len - zq < m) amb = 1;
                double php = wedge_angle(&w, a), ph = wedge_angle(&w, b);
                if (!(php > 0 && php < w.n * M_PI && ph > 0 && ph < w.n * M_PI)) ok = 0;
                if (php < 1e-4 || fabs(php - w.n * M_PI) < 1e-4 || ph < 1e-4 || fabs(ph - w.n * M_PI) < 1e-4) amb = 1;
            }
            if (ok && !(vlen(vsub(Q, b)) <= diff_max_leg)) ok = 0;
            v3 P = Q;
            if (ok) {  /* reflection point on the segment Q -> image */
                v3 img = rd ? a : b;
                v3 dv = vsub(img, Q);
                double den = vdot(n, dv);
                if (den == 0.0) ok = 0;
                double tt = ok ? (dpl - vdot(n, Q)) / den : 0.0;
                if (ok && !(tt > 0.0 && tt < 1.0)) ok = 0;
                if (ok && (tt < 1e-9 || tt > 1 - 1e-9)) amb = 1;
                P = vadd(Q, vmul(dv, tt));
            }
            if (ok) {
                int32_t found = -1;
                double ed = 0;
                for (int32_t j = face_off[f]; j < face_off[f + 1]; j++) {
                    int32_t t = face_tris[j];
                    double e1;
                    if (in_tri(P, tvert(tv, t, 0), tvert(tv, t, 1), tvert(tv, t, 2), &e1)) {
                        if (found < 0 || t < found) { found = t; ed = e1; }
                    }
                }
                if (found < 0) ok = 0;
                else {
                    if (ed < 1e-6) amb = 1;
                    tri_ids[5 * q + (rd ? 0 : 1)] = found;
                }
            }
            if (ok) {
                v3 x1 = rd ? P : Q, x2 = rd ? Q : P;
                points[15 * q + 0] = x1.x; points[15 * q + 1] = x1.y; points[15 * q + 2] = x1.z;
                points[15 * q + 3] = x2.x; points[15 * q + 4] = x2.y; points[15 * q + 5] = x2.z;
                if (rd) {
                    if (occluded(T, tv, tri_face, s, P, f, -1, &amb)) ok = 0;
                    else if (occluded3(T, tv, tri_face, P, Q, f, w.f0, w.fn, &amb)) ok = 0;
                    else if (occluded(T, tv, tri_face, Q, r, w.f0, w.fn, &amb)) ok = 0;
                } else {
                    if (occluded(T, tv, tri_face, s, Q, w.f0, w.fn, &amb)) ok = 0;
                    else if (occluded3(T, tv, tri_face, Q, P, w.f0, w.fn, f, &amb)) ok = 0;
                    else if (occluded(T, tv, tri_face, P, r, f, -1, &amb)) ok = 0;
                }
            }
        } else {
            ok = 0;
        }
        valid[q] = (uint8_t)ok;
        ambiguous[q] = (uint8_t)amb;
    }
    return n_bad;
}

/* Interaction points of fixed keys (the gradient reading: the topology is
 * held fixed, so containment, parameter ranges and occlusion are not
 * re-evaluated).  Specular: images s_k = mirror(s_{k-1}, plane f_k), then
 * back from Rx, x_k = segment(x_{k+1} -> s_k) meets plane f_k.  Diffraction:
 * the Keller point on the edge line, z_Q = z_s + (z_r - z_s) rho_s /
 * (rho_s + rho_r).  Line of sight has no points.  points [n][5][3]. */
int32_t orc_image_points(int32_t n_keys, const int32_t* keys, int32_t F, int32_t E, int32_t n_tx, int32_t n_rx,
                         const double* plane, const float* verts, const int32_t* edges, const double* edge_n,
                         const double* txp, const double* rxp, double* points) {
    int32_t n_bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_bad)
    for (int32_t q = 0; q < n_keys; q++) {
        const int32_t* key = keys + 9 * q;
        for (int i = 0; i < 15; i++) points[15 * q + i] = 0.0;
        if (!key_ok(key, n_tx, n_rx, F, E)) {  /* malformed: no points */
            n_bad++;
            continue;
        }
        v3 s = ld3d(txp + 3 * key[0]);
        v3 r = ld3d(rxp + 3 * key[1]);
        int type = key[2], order = key[3];
        if (type == 1) {
            v3 img[6];
            img[0] = s;
            for (int i = 1; i <= order; i++) {
                int32_t f = key[3 + i];
                img[i] = mirror(img[i - 1], ld3d(plane + 4 * f), plane[4 * f + 3]);
            }
            v3 cur = r;
            for (int i = order; i >= 1; i--) {
                int32_t f = key[3 + i];
                v3 n = ld3d(plane + 4 * f);
                v3 dv = vsub(img[i], cur);
                double tt = (plane[4 * f + 3] - vdot(n, cur)) / vdot(n, dv);
                cur = vadd(cur, vmul(dv, tt));
                points[15 * q + 3 * (i - 1) + 0] = cur.x;
                points[15 * q + 3 * (i - 1) + 1] = cur.y;
                points[15 * q + 3 * (i - 1) + 2] = cur.z;
            }
        } else if (type == 2) {
            orc_wedge w = wedge_at(verts, edges + 6 * key[4], edge_n[key[4]]);
            double zs = vdot(vsub(s, w.P0), w.e), zr = vdot(vsub(r, w.P0), w.e);
            double rs = vlen(vsub(vsub(s, w.P0), vmul(w.e, zs)));
            double rr = vlen(vsub(vsub(r, w.P0), vmul(w.e, zr)));
            double zq = zs + (zr - zs) * rs / (rs + rr);
            v3 Q = vadd(w.P0, vmul(w.e, zq));
            points[15 * q + 0] = Q.x;
            points[15 * q + 1] = Q.y;
            points[15 * q + 2] = Q.z;
        } else if (type == 3 || type == 4) {
            const int rd = type == 3;
            int32_t f = rd ? key[4] : key[5], e = rd ? key[5] : key[4];
            orc_wedge w = wedge_at(verts, edges + 6 * e, edge_n[e]);
            v3 n = ld3d(plane + 4 * f);
            double dpl = plane[4 * f + 3];
            v3 a = rd ? mirror(s, n, dpl) : s, b = rd ? r : mirror(r, n, dpl);
            double za = vdot(vsub(a, w.P0), w.e), zb = vdot(vsub(b, w.P0), w.e);
            double ra = vlen(vsub(vsub(a, w.P0), vmul(w.e, za)));
            double rb = vlen(vsub(vsub(b, w.P0), vmul(w.e, zb)));
            v3 Q = vadd(w.P0, vmul(w.e, za + (zb - za) * ra / (ra + rb)));
            v3 dv = vsub(rd ? a : b, Q);
            v3 P = vadd(Q, vmul(dv, (dpl - vdot(n, Q)) / vdot(n, dv)));
            v3 x1 = rd ? P : Q, x2 = rd ? Q : P;
            points[15 * q + 0] = x1.x; points[15 * q + 1] = x1.y; points[15 * q + 2] = x1.z;
            points[15 * q + 3] = x2.x; points[15 * q + 4] = x2.y; points[15 * q + 5] = x2.z;
        }
    }
    return n_bad;
}

/* ------------------------------------------------------------------------ */
/* fields                                                                    */
/* ------------------------------------------------------------------------ */

/* Fresnel reflection coefficients for a half space of complex relative
 * permittivity eps (eps' - j eps'', time factor exp(+j w t)) at incidence
 * cosine c (reading; the paper's Table I gives constant magnitudes, the
 * workloads give complex permittivities):
 *   Gamma_TE = (c - sqrt(eps - s^2)) / (c + sqrt(eps - s^2))
 *   Gamma_TM = (eps c - sqrt(eps - s^2)) / (eps c + sqrt(eps - s^2))
 * with s^2 = 1 - c^2 and the principal square root. */
void orc_fresnel_gamma(double er, double ei, double c, double* out) {
    double complex eps = er + I * ei;
    double s2 = 1.0 - c * c;
    double complex rt = csqrt(eps - s2);
    double complex te = (c - rt) / (c + rt);
    double complex tm = (eps * c - rt) / (eps * c + rt);
    out[0] = creal(te); out[1] = cimag(te); out[2] = creal(tm); out[3] = cimag(tm);
}

static void gammas(double complex eps, double c, double complex* te, double complex* tm) {
    double s2 = 1.0 - c * c;
    double complex rt = csqrt(eps - s2);
    *te = (c - rt) / (c + rt);
    *tm = (eps * c - rt) / (eps * c + rt);
}

/* Reflection coefficients of material m.  Table I lists surfaces by a
 * reflection coefficient alone (0.8 wall, 0.9 metal).  Reading: where
 * refl[m] = g > 0 the coefficient has magnitude g at every angle and for both
 * polarisations, with the signs a perfect conductor has in the basis above
 * (the eps -> infinity limit of the Fresnel forms: Gamma_TE = -g,
 * Gamma_TM = +g); refl[m] = 0 selects the Fresnel coefficients of the
 * material's permittivity. */
static void material_gammas(const double* mat_eps, const double* refl, int32_t m, double c, double complex* te,
                            double complex* tm) {
    if (refl[m] > 0.0) {
        *te = -refl[m];
        *tm = refl[m];
        return;
    }
    gammas(mat_eps[2 * m] + I * mat_eps[2 * m + 1], c, te, tm);
}

/* Scaled complementary error function erfcx(w) = exp(w^2) erfc(w) on the
 * ray w = exp(j pi/4) v, v >= 0.  Method: power series of erf
 * (Abramowitz & Stegun 7.1.5) for v < 2.5 and the Laplace continued
 * fraction (A&S 7.1.14) evaluated by the modified Lentz algorithm for
 * v >= 2.5. */
static double complex erfcx_diag(double v) {
    double complex w = v * cexp(I * M_PI / 4.0);
    if (v < 2.5) {
        double complex w2 = w * w;
        double complex term = w, sum = w;
        for (int n = 1; n < 400; n++) {
            term = term * (-w2) / (double)n;
            double complex add = term / (double)(2 * n + 1);
            sum += add;
            if (cabs(add) < 1e-18 * (cabs(sum) + 1e-300)) break;
        }
        double complex erfc_w = 1.0 - (2.0 / sqrt(M_PI)) * sum;
        return cexp(w2) * erfc_w;
    }
    /* K = w + a1/(w + a2/(w + ...)), a_n = n/2; erfcx = 1/(sqrt(pi) K) */
    const double tiny = 1e-300;
    double complex f = w, C = w, D = 0.0;
    for (int n = 1; n < 5000; n++) {
        double an = 0.5 * n;
        D = w + an * D;
        if (cabs(D) < tiny) D = tiny;
        C = w + an / C;
        if (cabs(C) < tiny) C = tiny;
        D = 1.0 / D;
        double complex delta = C * D;
        f *= delta;
        if (cabs(delta - 1.0) < 1e-16) break;
    }
    return 1.0 / (sqrt(M_PI) * f);
}

/* UTD transition function F(X) = 2j sqrt(X) e^{jX} int_{sqrt X}^inf
 * e^{-j tau^2} d tau (Kouyoumjian & Pathak 1974), X >= 0, written as
 * F(X) = e^{j pi/4} sqrt(pi X) erfcx(e^{j pi/4} sqrt X). */
static double complex utd_F(double X) {
    if (X <= 0) return 0.0;
    double v = sqrt(X);
    return cexp(I * M_PI / 4.0) * sqrt(M_PI * X) * erfcx_diag(v);
}

void orc_utd_F(double X, double* out) {
    double complex f = utd_F(X);
    out[0] = creal(f); out[1] = cimag(f);
}

void orc_erfcx_diag(double v, double* out) {
    double complex f = erfcx_diag(v);
    out[0] = creal(f); out[1] = cimag(f);
}

/* One cotangent term of the UTD coefficient:
 * cot((pi + sg*beta)/(2n)) F(kL a^{sg}(beta)),
 * a^{+-}(beta) = 2 cos^2((2 n pi N^{+-} - beta)/2), N^{+-} the integer
 * nearest (beta +- pi)/(2 pi n).  Within |eps| < 1e-4 of the shadow or
 * reflection boundary (eps = pi + sg(beta - 2 pi n N)) the small-argument
 * limit n e^{j pi/4} [sqrt(2 pi kL) sgn(eps) - 2 kL eps e^{j pi/4}] is used
 * (reading: the cot * F product is finite there but 0 * inf numerically). */
static double complex utd_term(double sg, double beta, double n, double kL) {
    double N = round((beta + sg * M_PI) / (2.0 * M_PI * n));
    double eps = M_PI + sg * (beta - 2.0 * M_PI * n * N);
    if (fabs(eps) < 1e-4) {
        double sgn = eps > 0 ? 1.0 : (eps < 0 ? -1.0 : 0.0);
        double complex e4 = cexp(I * M_PI / 4.0);
        return n * e4 * (sqrt(2.0 * M_PI * kL) * sgn - 2.0 * kL * eps * e4);
    }
    double c = cos((2.0 * M_PI * n * N - beta) / 2.0);
    double a = 2.0 * c * c;
    double x = (M_PI + sg * beta) / (2.0 * n);
    return (cos(x) / sin(x)) * utd_F(kL * a);
}

/* Diffraction coefficients D_s (soft) and D_h (hard) of a wedge with exterior
 * angle n pi: Kouyoumjian-Pathak (1974) with the Luebbers (1984) lossy-face
 * form, D = C [T(+,phi-phi') + T(-,phi-phi') + R_n T(+,phi+phi') +
 * R_0 T(-,phi+phi')], C = -e^{-j pi/4} / (2 n sqrt(2 pi k) sin beta0).
 * R_0 / R_n are the reflection coefficients (material_gammas) of the 0-face /
 * n-face materials m0 / mn (TE for soft, TM for hard) at incidence cosines
 * sin(beta0) |sin phi'| and
 * sin(beta0) |sin(n pi - phi)| (reading: Luebbers' grazing angles, taken on
 * the actual incidence angle for an oblique edge). */
static void utd_D(double n, double k, double L, double beta0, double php, double ph, const double* mat_eps,
                  const double* refl, int32_t m0, int32_t mn, double complex* Ds, double complex* Dh) {
    double sb = sin(beta0);
    double complex C = -cexp(-I * M_PI / 4.0) / (2.0 * n * sqrt(2.0 * M_PI * k) * sb);
    double kL = k * L;
    double complex t1 = utd_term(+1, ph - php, n, kL);
    double complex t2 = utd_term(-1, ph - php, n, kL);
    double complex t3 = utd_term(+1, ph + php, n, kL);
    double complex t4 = utd_term(-1, ph + php, n, kL);
    double c0 = sb * fabs(sin(php));
    double cn = sb * fabs(sin(n * M_PI - ph));
    double complex r0te, r0tm, rnte, rntm;
    material_gammas(mat_eps, refl, m0, c0, &r0te, &r0tm);
    material_gammas(mat_eps, refl, mn, cn, &rnte, &rntm);
    *Ds = C * (t1 + t2 + rnte * t3 + r0te * t4);
    *Dh = C * (t1 + t2 + rntm * t3 + r0tm * t4);
}

void orc_utd_D(double n, double k, double L, double beta0, double php, double ph, const double* eps0,
               const double* epsn, double* out) {
    double complex ds, dh;
    const double mats[4] = {eps0[0], eps0[1], epsn[0], epsn[1]}, refl[2] = {0.0, 0.0};
    utd_D(n, k, L, beta0, php, ph, mats, refl, 0, 1, &ds, &dh);
    out[0] = creal(ds); out[1] = cimag(ds); out[2] = creal(dh); out[3] = cimag(dh);
}

/* Antenna polarisation vector for propagation direction k (reading of
 * Section IV's "ideal and omnidirectional" antenna): mode 0 (vertical iso):
 * e = normalize(z - (z.k) k), x used instead of z when k is along z; gain 1.
 * Mode 1 (short dipole along u(theta, phi)): e = sqrt(1.5) (u - (u.k) k). */
static v3 antenna(int mode, v3 k, double th, double ph) {
    if (mode == 1) {
        v3 u = V(sin(th) * cos(ph), sin(th) * sin(ph), cos(th));
        return vmul(vsub(u, vmul(k, vdot(u, k))), sqrt(1.5));
    }
    v3 z = V(0, 0, 1);
    v3 e = vsub(z, vmul(k, vdot(z, k)));
    if (vlen(e) < 1e-12) { v3 x = V(1, 0, 0); e = vsub(x, vmul(k, vdot(x, k))); }
    return vnorm(e);
}

typedef struct { double complex x, y, z; } c3;
static double complex cdotr(v3 a, c3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static c3 cmk(v3 a, double complex s) { c3 r = {a.x * s, a.y * s, a.z * s}; return r; }
static c3 cadd(c3 a, c3 b) { c3 r = {a.x + b.x, a.y + b.y, a.z + b.z}; return r; }

/* Reflect the field vector E travelling along ki into ko at face f: the s/p
 * basis of the bounce (s = normalize(ki x n), n against ki; normal incidence
 * n x z, else n x x), E <- Gamma_TE (E.s) s + Gamma_TM (E.p_in) p_out. */
static c3 reflect_at(c3 E, v3 ki, v3 ko, int32_t f, const double* plane, const int32_t* face_material,
                     const double* mat_eps, const double* mat_refl) {
    v3 n = ld3d(plane + 4 * f);
    if (vdot(n, ki) > 0) n = vmul(n, -1.0);
    double c = -vdot(ki, n);
    v3 sv = vcross(ki, n);
    if (vlen(sv) < 1e-12) {
        sv = vcross(n, V(0, 0, 1));
        if (vlen(sv) < 1e-12) sv = vcross(n, V(1, 0, 0));
    }
    sv = vnorm(sv);
    v3 pin = vcross(sv, ki), pout = vcross(sv, ko);
    double complex te, tm;
    material_gammas(mat_eps, mat_refl, face_material[f], c, &te, &tm);
    double complex es = cdotr(sv, E), ep = cdotr(pin, E);
    return cadd(cmk(sv, te * es), cmk(pout, tm * ep));
}

/* phase factor exp(-j 2 pi frac(L / lambda)), frac(x) = x - round(x) */
static double complex phase(double L, double lam) {
    double x = L / lam;
    double fr = x - round(x);
    return cexp(-I * 2.0 * M_PI * fr);
}

/* Field evaluation of validated paths (double precision throughout).
 *   Specular, order K with points x_1..x_K: E = e_tx(k_0); at bounce i with
 *   incident k_{i-1}, outgoing k_i and face normal n oriented against k_{i-1}:
 *   s = normalize(k_{i-1} x n) (normal incidence: normalize(n x z), else
 *   normalize(n x x)), p_in = s x k_{i-1}, p_out = s x k_i,
 *   E <- Gamma_TE (E.s) s + Gamma_TM (E.p_in) p_out, with the coefficients of
 *   the face's material (material_gammas: Fresnel from mat_eps [M][2], or the
 *   constant magnitude mat_refl [M] where that is > 0);
 *   a = lambda/(4 pi L) (e_rx(k_K).E) exp(-j 2 pi frac(L/lambda)), L the
 *   unfolded length (line of sight: Friis amplitude).
 *   Diffraction: a = lambda/(4 pi) (1/s') sqrt(s'/(s (s+s'))) e_rx.(D.e_tx)
 *   exp(-j 2 pi frac((s+s')/lambda)), dyadic D = -b0 b0' D_s - ph ph' D_h
 *   with ph' = -normalize(e x s_in), b0' = ph' x s_in, ph = normalize(e x
 *   s_out), b0 = ph x s_out.
 *   Delay tau = L / c.  Doppler (Section III-C, Eq (3) generalised to moving
 *   interaction points, reading): f_D = -(1/lambda) [k_K.v_rx - k_0.v_tx +
 *   sum_i (k_{i-1} - k_i).v_obj(i)], v_obj the translational velocity of the
 *   object owning face / edge i; for line of sight with a static base
 *   station this is Eq (3) exactly.
 *   AoD = (azimuth, elevation) of k_0, AoA = (azimuth, elevation) of -k_K.
 * Outputs: a [n][nf][2], tau [n], fd [n][nf], aod [n][2], aoa [n][2]. */
int32_t orc_eval(int32_t n_paths, const int32_t* keys, int32_t F, int32_t E, int32_t n_tx, int32_t n_rx,
                 const double* points, const double* plane,
                 const int32_t* face_material, const int32_t* face_dyn, const double* obj_vel,
                 const double* mat_eps, const double* mat_refl, const float* verts, const int32_t* edges,
                 const double* edge_n,
                 const double* txp, const double* txv, const double* txo, const double* rxp, const double* rxv,
                 int32_t ant_mode, int32_t nf, const double* freqs,
                 double* a_out, double* tau_out, double* fd_out, double* aod, double* aoa) {
    int32_t n_bad = 0;
    if (nf < 1 || nf > 8) return -1;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n_bad)
    for (int32_t q = 0; q < n_paths; q++) {
        const int32_t* key = keys + 9 * q;
        if (!key_ok(key, n_tx, n_rx, F, E)) {  /* malformed: NaN outputs */
            for (int fi = 0; fi < nf; fi++) {
                a_out[2 * (q * nf + fi)] = a_out[2 * (q * nf + fi) + 1] = NAN;
                fd_out[q * nf + fi] = NAN;
            }
            tau_out[q] = aod[2 * q] = aod[2 * q + 1] = aoa[2 * q] = aoa[2 * q + 1] = NAN;
            n_bad++;
            continue;
        }
        int tx = key[0], rx = key[1], type = key[2], order = key[3];
        v3 s = ld3d(txp + 3 * tx), r = ld3d(rxp + 3 * rx);
        v3 vt = ld3d(txv + 3 * tx), vr = ld3d(rxv + 3 * rx);
        double th = txo[2 * tx], phi = txo[2 * tx + 1];
        v3 k0, kK;
        double L = 0.0, dop = 0.0; /* dop = dL/dt */
        double complex amp[8];
        if (type == 0 || type == 1) {
            v3 P[7];
            int np = 0;
            P[np++] = s;
            if (type == 1)
                for (int i = 0; i < order; i++) P[np++] = ld3d(points + 15 * q + 3 * i);
            P[np++] = r;
            v3 kk[7];
            for (int i = 0; i + 1 < np; i++) {
                v3 dv = vsub(P[i + 1], P[i]);
                double l = vlen(dv);
                L += l;
                kk[i] = vmul(dv, 1.0 / l);
            }
            k0 = kk[0];
            kK = kk[np - 2];
            dop = vdot(kK, vr) - vdot(k0, vt);
            for (int i = 1; i + 1 < np; i++) {
                int32_t f = key[3 + i];
                int32_t od = face_dyn[f];
                if (od >= 0) dop += vdot(vsub(kk[i - 1], kk[i]), ld3d(obj_vel + 3 * od));
            }
            for (int fi = 0; fi < nf; fi++) {
                double lam = ORC_C0 / freqs[fi];
                v3 e0 = antenna(ant_mode, k0, th, phi);
                c3 E = cmk(e0, 1.0);
                for (int i = 1; i + 1 < np; i++)
                    E = reflect_at(E, kk[i - 1], kk[i], key[3 + i], plane, face_material, mat_eps, mat_refl);
                v3 er = antenna(0, kK, 0, 0);
                amp[fi] = lam / (4.0 * M_PI * L) * cdotr(er, E) * phase(L, lam);
            }
        } else {
            /* diffraction alone (2), after a reflection (3) or before one (4):
             * points s, [P], Q, [P], r; the reflection at P acts on the field
             * vector arriving at Q (3) or leaving it (4); the spreading uses the
             * unfolded source-side and receiver-side lengths. */
            const int rd = type == 3, dr = type == 4;
            int32_t e = rd ? key[5] : key[4];
            int32_t fr = rd ? key[4] : (dr ? key[5] : -1);
            orc_wedge w = wedge_at(verts, edges + 6 * e, edge_n[e]);
            v3 X1 = ld3d(points + 15 * q), X2 = ld3d(points + 15 * q + 3);
            v3 Q = rd ? X2 : X1, Pr = rd ? X1 : X2;
            v3 pt[4];
            int np = 0;
            pt[np++] = s;
            if (rd) pt[np++] = Pr;
            pt[np++] = Q;
            if (dr) pt[np++] = Pr;
            pt[np++] = r;
            v3 kk[3];
            double seg[3];
            for (int i = 0; i + 1 < np; i++) {
                v3 dv = vsub(pt[i + 1], pt[i]);
                seg[i] = vlen(dv);
                kk[i] = vmul(dv, 1.0 / seg[i]);
                L += seg[i];
            }
            const int iq = rd ? 1 : 0; /* segment arriving at Q */
            v3 si = kk[iq], so = kk[iq + 1];
            double sp = rd ? seg[0] + seg[1] : seg[0];
            double sd = dr ? seg[1] + seg[2] : seg[iq + 1];
            k0 = kk[0];
            kK = kk[np - 2];
            dop = vdot(kK, vr) - vdot(k0, vt);
            int32_t od = face_dyn[w.f0];
            if (od >= 0) dop += vdot(vsub(si, so), ld3d(obj_vel + 3 * od));
            if (fr >= 0) {
                int32_t of = face_dyn[fr];
                int ip = rd ? 1 : 2; /* point index of P: the segments ip - 1 and ip meet there */
                if (of >= 0) dop += vdot(vsub(kk[ip - 1], kk[ip]), ld3d(obj_vel + 3 * of));
            }
            double cb = vdot(si, w.e);
            if (cb > 1) cb = 1;
            if (cb < -1) cb = -1;
            double beta0 = acos(cb);
            double php = wedge_angle(&w, pt[iq]), ph = wedge_angle(&w, pt[iq + 2]);
            double Lp = sd * sp * sin(beta0) * sin(beta0) / (sd + sp);
            v3 fp = vmul(vnorm(vcross(w.e, si)), -1.0), bp = vcross(fp, si);
            v3 fo = vnorm(vcross(w.e, so)), bo = vcross(fo, so);
            int32_t m0 = face_material[w.f0], mn = face_material[w.fn];
            for (int fi = 0; fi < nf; fi++) {
                double lam = ORC_C0 / freqs[fi];
                double k = 2.0 * M_PI / lam;
                double complex Ds, Dh;
                utd_D(w.n, k, Lp, beta0, php, ph, mat_eps, mat_refl, m0, mn, &Ds, &Dh);
                c3 E = cmk(antenna(ant_mode, k0, th, phi), 1.0);
                if (rd) E = reflect_at(E, kk[0], kk[1], fr, plane, face_material, mat_eps, mat_refl);
                c3 Ed = cadd(cmk(bo, -cdotr(bp, E) * Ds), cmk(fo, -cdotr(fp, E) * Dh));
                if (dr) Ed = reflect_at(Ed, kk[1], kk[2], fr, plane, face_material, mat_eps, mat_refl);
                v3 er = antenna(0, kK, 0, 0);
                amp[fi] = lam / (4.0 * M_PI) * (1.0 / sp) * sqrt(sp / (sd * (sd + sp))) * cdotr(er, Ed) * phase(L, lam);
            }
        }
        for (int fi = 0; fi < nf; fi++) {
            double lam = ORC_C0 / freqs[fi];
            a_out[2 * (q * nf + fi)] = creal(amp[fi]);
            a_out[2 * (q * nf + fi) + 1] = cimag(amp[fi]);
            fd_out[q * nf + fi] = -dop / lam;
        }
        tau_out[q] = L / ORC_C0;
        aod[2 * q] = atan2(k0.y, k0.x);
        aod[2 * q + 1] = asin(k0.z > 1 ? 1 : (k0.z < -1 ? -1 : k0.z));
        aoa[2 * q] = atan2(-kK.y, -kK.x);
        aoa[2 * q + 1] = asin(-kK.z > 1 ? 1 : (-kK.z < -1 ? -1 : -kK.z));
    }
    return n_bad;
}

int32_t orc_num_threads(void) { return omp_get_max_threads(); }
