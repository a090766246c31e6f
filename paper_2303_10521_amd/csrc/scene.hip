// scene.hip -- scene ingest and per-frame geometry.
//
// Once per scene: index checks, dynamic-object ranks, face -> triangle lists,
// static / dynamic triangle partitions and the wedge edges used for
// first-order diffraction (Section II-A names diffracted rays; the edge model
// is this library's reading: convex edges where two faces of one object meet).
// Every frame: world vertices of the moving objects (Section III-A moving
// objects, rigid transforms supplied per frame), face planes in double, and
// the primitive boxes the LBVH builds over.
#include "emrt_dev.h"
#include "emrt_launch.h"

namespace emrt {

static int grid_for(long long n, int block = 256) {
    long long g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65535 * 4) g = 65535 * 4;
    return (int)g;
}

#define GRID_STRIDE(i, n) for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

__global__ void k_check(int V, int T, int F, int O, int M, const int* tris, const int* tri_face,
                        const int* face_object, const int* face_material, const float* verts, uint32_t* flags) {
    GRID_STRIDE(i, (long long)T) {
        bool bad = false;
        for (int k = 0; k < 3; k++) {
            int v = tris[3 * i + k];
            if (v < 0 || v >= V) bad = true;
        }
        int f = tri_face[i];
        if (f < 0 || f >= F) bad = true;
        if (!bad) {
            const float* a = verts + 3 * tris[3 * i];
            const float* b = verts + 3 * tris[3 * i + 1];
            const float* c = verts + 3 * tris[3 * i + 2];
            dv3 e1 = d3((double)b[0] - a[0], (double)b[1] - a[1], (double)b[2] - a[2]);
            dv3 e2 = d3((double)c[0] - a[0], (double)c[1] - a[1], (double)c[2] - a[2]);
            if (!(len(cross(e1, e2)) > 0.0)) bad = true;
            for (int k = 0; k < 3; k++)
                if (!isfinite(a[k]) || !isfinite(b[k]) || !isfinite(c[k])) bad = true;
        }
        if (bad) atomicOr(flags, FLAG_BAD_INPUT);
    }
    GRID_STRIDE(i, (long long)F) {
        int o = face_object[i], m = face_material[i];
        if (o < 0 || o >= O || m < 0 || m >= M) atomicOr(flags, FLAG_BAD_INPUT);
    }
}

__global__ void k_u8_to_u32(const uint8_t* in, uint32_t* out, long long n) {
    GRID_STRIDE(i, n) out[i] = in[i] ? 1u : 0u;
}

__global__ void k_ranks(const uint8_t* dyn, const uint32_t* scan, int O, int* obj_rank) {
    GRID_STRIDE(i, (long long)O) obj_rank[i] = dyn[i] ? (int)scan[i] : -1;
}

__global__ void k_face_setup(int F, const int* face_object, const int* obj_rank, int* face_dyn, int* face_first,
                             uint32_t* face_count) {
    GRID_STRIDE(i, (long long)F) {
        face_dyn[i] = obj_rank[face_object[i]];
        face_first[i] = 0x7FFFFFFF;
        face_count[i] = 0;
    }
}

__global__ void k_tri_setup(int T, const int* tris, const int* tri_face, const int* face_dyn, int* vert_dyn,
                            int* face_first, uint32_t* face_count, uint32_t* is_static,
                            unsigned long long* keys, uint32_t* vals) {
    GRID_STRIDE(i, (long long)T) {
        int f = tri_face[i];
        int d = face_dyn[f];
        for (int k = 0; k < 3; k++) vert_dyn[tris[3 * i + k]] = d;
        atomicMin(&face_first[f], (int)i);
        atomicAdd(&face_count[f], 1u);
        is_static[i] = d < 0 ? 1u : 0u;
        keys[i] = ((unsigned long long)(uint32_t)f << 32) | (uint32_t)i;
        vals[i] = (uint32_t)i;
    }
}

__global__ void k_partition(int T, const uint32_t* is_static, const uint32_t* pos, int* st_list, int* dy_list) {
    GRID_STRIDE(i, (long long)T) {
        uint32_t p = pos[i];
        if (is_static[i]) st_list[p] = (int)i;
        else dy_list[i - p] = (int)i;
    }
}

__global__ void k_copy_i32(const uint32_t* in, int* out, long long n) {
    GRID_STRIDE(i, n) out[i] = (int)in[i];
}

__global__ void k_copy_f32(const float* in, float* out, long long n) {
    GRID_STRIDE(i, n) out[i] = in[i];
}

__global__ void k_count_total(const uint32_t* scan_last, const uint32_t* last_flag, long long n, int* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = n > 0 ? (int)(scan_last[0] + last_flag[0]) : 0;
}

void scene_check(const SceneDev& s, const uint8_t* object_dynamic, uint32_t* flags, hipStream_t st) {
    (void)object_dynamic;
    hipLaunchKernelGGL(k_check, dim3(grid_for(s.T > s.F ? s.T : s.F)), dim3(256), 0, st, s.V, s.T, s.F, s.O, s.M,
                       s.tris, s.tri_face, s.face_object, s.face_material, s.verts_local_copy, flags);
}

// scratch_u32 must hold 4 * max(T, O, F) + scan temp; counts_dev gets
// [O_d, T_s] on return (device ints).
void scene_prepare(SceneDev& s, const uint8_t* object_dynamic, uint32_t* scratch_u32, int* counts_dev,
                   const BuildTemp& tmp, hipStream_t st) {
    long long big = s.T;
    if (s.O > big) big = s.O;
    if (s.F > big) big = s.F;
    uint32_t* a = scratch_u32;
    uint32_t* b = a + big;
    uint32_t* c = b + big;
    uint32_t* stemp = c + big + 16;
    // dynamic ranks
    hipLaunchKernelGGL(k_u8_to_u32, dim3(grid_for(s.O)), dim3(256), 0, st, object_dynamic, a, (long long)s.O);
    exclusive_scan(a, b, s.O, stemp, (uint32_t*)&counts_dev[0], st);
    hipLaunchKernelGGL(k_ranks, dim3(grid_for(s.O)), dim3(256), 0, st, object_dynamic, b, s.O, s.obj_rank);
    // faces
    hipLaunchKernelGGL(k_face_setup, dim3(grid_for(s.F)), dim3(256), 0, st, s.F, s.face_object, s.obj_rank,
                       s.face_dyn, s.face_first, a);
    fill_u32((uint32_t*)s.vert_dyn, 0xFFFFFFFFu, s.V, st);
    hipLaunchKernelGGL(k_tri_setup, dim3(grid_for(s.T)), dim3(256), 0, st, s.T, s.tris, s.tri_face, s.face_dyn,
                       s.vert_dyn, s.face_first, a, c, tmp.k0, tmp.v0);
    // face -> triangles (sorted by (face, tri))
    exclusive_scan(a, (uint32_t*)s.face_off, s.F, stemp, (uint32_t*)&s.face_off[s.F], st);
    int which = radix_sort(tmp.k0, tmp.v0, tmp.k1, tmp.v1, nullptr, s.T, 64, tmp.radix, st);
    hipLaunchKernelGGL(k_copy_i32, dim3(grid_for(s.T)), dim3(256), 0, st, which ? tmp.v1 : tmp.v0, s.face_tris,
                       (long long)s.T);
    // static / dynamic partitions, order by triangle id
    exclusive_scan(c, b, s.T, stemp, (uint32_t*)&counts_dev[1], st);
    hipLaunchKernelGGL(k_partition, dim3(grid_for(s.T)), dim3(256), 0, st, s.T, c, b, s.tris_static,
                       s.tris_dynamic);
}

// ------------------------------------------------------------- edges ----
// Wedge edges of one object (reading; the paper names diffracted rays, not an
// edge model): for each pair of non-parallel faces f < g of the object, the
// triangle edges of f lying on plane g and those of g lying on plane f (both
// ends within 1 mm) lie on the two planes' intersection line; the overlap of
// their extents along u = normalize(n_f x n_g) is the edge.  Kept when convex
// seen from outside (triangles wound counter-clockwise from outside): the
// in-face direction t_n of g satisfies t_n . n_f < 0.  The exterior angle is
// n pi, n = atan2(t_n . n_f, t_n . t_0) / pi in (1, 2).
__device__ __forceinline__ dv3 plane_local(const SceneDev& s, int f, double& d) {
    int t = s.face_first[f];
    dv3 a = ldf3(s.verts_local_copy + 3 * s.tris[3 * t]);
    dv3 b = ldf3(s.verts_local_copy + 3 * s.tris[3 * t + 1]);
    dv3 c = ldf3(s.verts_local_copy + 3 * s.tris[3 * t + 2]);
    dv3 n = unit(cross(b - a, c - a));
    d = dot(n, a);
    return n;
}

__global__ void k_obj_faces_setup(int F, const int* face_object, uint32_t* cnt, unsigned long long* keys,
                                  uint32_t* vals) {
    GRID_STRIDE(i, (long long)F) {
        int o = face_object[i];
        atomicAdd(&cnt[o], 1u);
        keys[i] = ((unsigned long long)(uint32_t)o << 32) | (uint32_t)i;
        vals[i] = (uint32_t)i;
    }
}

__global__ void k_edges(SceneDev s, const int* obj_off, const int* obj_faces, int* counter, int cap,
                        unsigned long long* keys, uint32_t* vals, int* rows, double* wn) {
    GRID_STRIDE(o, (long long)s.O) {
        int f_beg = obj_off[o], f_end = obj_off[o + 1];
        for (int ia = f_beg; ia < f_end; ia++) {
            for (int ib = f_beg; ib < f_end; ib++) {
                int f = obj_faces[ia], g = obj_faces[ib];
                if (!(f < g)) continue;
                double df, dg;
                dv3 nf = plane_local(s, f, df), ng = plane_local(s, g, dg);
                dv3 u = cross(nf, ng);
                if (len(u) < 1e-6) continue;
                u = unit(u);
                const double tol = 1e-3;
                double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
                int vlo[2] = {-1, -1}, vhi[2] = {-1, -1};
                for (int side = 0; side < 2; side++) {
                    int ff = side ? g : f;
                    dv3 on = side ? nf : ng;
                    double od = side ? df : dg;
                    for (int q = s.face_off[ff]; q < s.face_off[ff + 1]; q++) {
                        int t = s.face_tris[q];
                        for (int k = 0; k < 3; k++) {
                            int va = s.tris[3 * t + k], vb = s.tris[3 * t + (k + 1) % 3];
                            dv3 pa = ldf3(s.verts_local_copy + 3 * va), pb = ldf3(s.verts_local_copy + 3 * vb);
                            if (fabs(dot(on, pa) - od) > tol || fabs(dot(on, pb) - od) > tol) continue;
                            if (len(pa - pb) < tol) continue;
                            double sa = dot(pa, u), sb = dot(pb, u);
                            if (sa < lo[side] || (sa == lo[side] && va < vlo[side])) { lo[side] = sa; vlo[side] = va; }
                            if (sb < lo[side] || (sb == lo[side] && vb < vlo[side])) { lo[side] = sb; vlo[side] = vb; }
                            if (sa > hi[side] || (sa == hi[side] && va < vhi[side])) { hi[side] = sa; vhi[side] = va; }
                            if (sb > hi[side] || (sb == hi[side] && vb < vhi[side])) { hi[side] = sb; vhi[side] = vb; }
                        }
                    }
                }
                if (vlo[0] < 0 || vlo[1] < 0) continue;
                double a0 = lo[0] > lo[1] ? lo[0] : lo[1];
                double a1 = hi[0] < hi[1] ? hi[0] : hi[1];
                if (!(a1 - a0 > tol)) continue;
                int va = lo[0] > lo[1] ? vlo[0] : (lo[1] > lo[0] ? vlo[1] : (vlo[0] < vlo[1] ? vlo[0] : vlo[1]));
                int vb = hi[0] < hi[1] ? vhi[0] : (hi[1] < hi[0] ? vhi[1] : (vhi[0] < vhi[1] ? vhi[0] : vhi[1]));
                dv3 P0 = ldf3(s.verts_local_copy + 3 * va);
                int w[2] = {-1, -1};
                for (int side = 0; side < 2; side++) {
                    int ff = side ? g : f;
                    double best = -1.0;
                    for (int q = s.face_off[ff]; q < s.face_off[ff + 1]; q++) {
                        int t = s.face_tris[q];
                        for (int k = 0; k < 3; k++) {
                            int vv = s.tris[3 * t + k];
                            dv3 r = ldf3(s.verts_local_copy + 3 * vv) - P0;
                            double dd = len(r - u * dot(r, u));
                            if (dd > best + 1e-12) { best = dd; w[side] = vv; }
                        }
                    }
                }
                dv3 r0 = ldf3(s.verts_local_copy + 3 * w[0]) - P0, rn = ldf3(s.verts_local_copy + 3 * w[1]) - P0;
                dv3 t0 = unit(r0 - u * dot(r0, u));
                dv3 tn = unit(rn - u * dot(rn, u));
                double yy = dot(tn, nf), xx = dot(tn, t0);
                if (!(yy < -1e-9)) continue;
                double phn = atan2(yy, xx);
                if (phn < 0) phn += 2.0 * kPi;
                int slot = atomicAdd(counter, 1);
                if (slot < cap) {
                    int* row = rows + 6 * (long long)slot;
                    row[0] = va; row[1] = vb; row[2] = f; row[3] = g; row[4] = w[0]; row[5] = w[1];
                    wn[slot] = phn / kPi;
                    keys[slot] = ((unsigned long long)(uint32_t)f << 32) | (uint32_t)g;
                    vals[slot] = (uint32_t)slot;
                }
            }
        }
    }
}

__global__ void k_edge_order(const uint32_t* order, int n, const int* rows, const double* wn, int* out_rows,
                             double* out_wn) {
    GRID_STRIDE(i, (long long)n) {
        uint32_t j = order[i];
        for (int k = 0; k < 6; k++) out_rows[6 * i + k] = rows[6 * (long long)j + k];
        out_wn[i] = wn[j];
    }
}

// obj_off: [O+1] ints, obj_faces: [F] ints, counter: device int.  Uses the
// build temp (k0/v0/k1/v1 of capacity >= max(F, E_cap)) and returns E (host).
int scene_edges(SceneDev& s, int* obj_off, int* obj_faces, int* counter, const BuildTemp& tmp, hipStream_t st) {
    uint32_t* cnt = (uint32_t*)obj_faces;  // reuse as counts before the faces are written
    fill_u32(tmp.v1, 0u, s.O + 1, st);
    hipLaunchKernelGGL(k_obj_faces_setup, dim3(grid_for(s.F)), dim3(256), 0, st, s.F, s.face_object, tmp.v1, tmp.k0,
                       tmp.v0);
    (void)cnt;
    exclusive_scan(tmp.v1, (uint32_t*)obj_off, s.O, (uint32_t*)tmp.radix, (uint32_t*)&obj_off[s.O], st);
    int which = radix_sort(tmp.k0, tmp.v0, tmp.k1, tmp.v1, nullptr, s.F, 64, tmp.radix, st);
    hipLaunchKernelGGL(k_copy_i32, dim3(grid_for(s.F)), dim3(256), 0, st, which ? tmp.v1 : tmp.v0, obj_faces,
                       (long long)s.F);
    // edge rows into a staging area behind the final arrays
    int* rows_stage = s.edge_i + 6 * (long long)s.E_cap;
    double* wn_stage = s.edge_n + s.E_cap;
    fill_u32((uint32_t*)counter, 0u, 1, st);
    hipLaunchKernelGGL(k_edges, dim3(grid_for(s.O, 64)), dim3(64), 0, st, s, obj_off, obj_faces, counter, s.E_cap,
                       tmp.k0, tmp.v0, rows_stage, wn_stage);
    int E = 0;
    hipError_t err = hipMemcpyAsync(&E, counter, sizeof(int), hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (err != hipSuccess) return -(1 << 30);
    if (E > s.E_cap) return -E;
    s.E = E;
    if (E > 0) {
        int w2 = radix_sort(tmp.k0, tmp.v0, tmp.k1, tmp.v1, nullptr, E, 64, tmp.radix, st);
        hipLaunchKernelGGL(k_edge_order, dim3(grid_for(E)), dim3(256), 0, st, w2 ? tmp.v1 : tmp.v0, E, rows_stage,
                           wn_stage, s.edge_i, s.edge_n);
    }
    return E;
}

// ---------------------------------------------------- per-frame geometry ----
// World vertex rule for moving objects: float32(((R0 x + R1 y) + R2 z) + t),
// evaluated in double without fused multiply-add.
__global__ void k_world(int V, const float* vloc, const int* vdyn, const double* xform, float* out, uint32_t* flags) {
#pragma clang fp contract(off)
    GRID_STRIDE(v, (long long)V) {
        int o = vdyn[v];
        if (o < 0) continue;
        const double* m = xform + 12 * (long long)o;
        double x = vloc[3 * v], y = vloc[3 * v + 1], z = vloc[3 * v + 2];
        for (int i = 0; i < 3; i++) {
            double a = __dmul_rn(m[4 * i + 0], x);
            double b = __dmul_rn(m[4 * i + 1], y);
            double c = __dmul_rn(m[4 * i + 2], z);
            double s = __dadd_rn(a, b);
            s = __dadd_rn(s, c);
            s = __dadd_rn(s, m[4 * i + 3]);
            if (!isfinite(s)) atomicOr(flags, FLAG_NONFINITE);
            out[3 * v + i] = (float)s;
        }
    }
}

void scene_world(const SceneDev& s, const double* xform, uint32_t* flags, hipStream_t st) {
    if (s.O_d <= 0) return;
    hipLaunchKernelGGL(k_world, dim3(grid_for(s.V)), dim3(256), 0, st, s.V, s.verts_local_copy, s.vert_dyn, xform,
                       s.verts, flags);
}

// Face plane: unit normal of the face's lowest-id triangle and n.v0, double.
__global__ void k_planes(int F, const int* face_first, const int* tris, const float* verts, double* plane) {
    GRID_STRIDE(f, (long long)F) {
        int t = face_first[f];
        dv3 a = ldf3(verts + 3 * tris[3 * t]);
        dv3 b = ldf3(verts + 3 * tris[3 * t + 1]);
        dv3 c = ldf3(verts + 3 * tris[3 * t + 2]);
        dv3 n = unit(cross(b - a, c - a));
        plane[4 * f + 0] = n.x;
        plane[4 * f + 1] = n.y;
        plane[4 * f + 2] = n.z;
        plane[4 * f + 3] = dot(n, a);
    }
}

void scene_planes(const SceneDev& s, hipStream_t st) {
    hipLaunchKernelGGL(k_planes, dim3(grid_for(s.F)), dim3(256), 0, st, s.F, s.face_first, s.tris, s.verts, s.plane);
}

__global__ void k_face_tv(int T, const int* face_tris, const int* tris, const float* verts, float* tv) {
    GRID_STRIDE(q, (long long)T) {
        int t = face_tris[q];
        for (int k = 0; k < 3; k++) {
            const float* v = verts + 3 * (long long)tris[3 * t + k];
            tv[9 * q + 3 * k] = v[0];
            tv[9 * q + 3 * k + 1] = v[1];
            tv[9 * q + 3 * k + 2] = v[2];
        }
    }
}

// bounding box of each face's triangles (after k_face_tv); only faces of at
// most 32 triangles use it (larger faces are searched through the LBVH)
__global__ void k_face_box(int F, const int* face_off, const float* tv, float* box) {
    GRID_STRIDE(f, (long long)F) {
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        int q0 = face_off[f], q1 = face_off[f + 1];
        if (q1 - q0 > 32) q1 = q0;  // box unused
        for (int q = q0; q < q1; q++)
            for (int k = 0; k < 9; k++) {
                float v = tv[9 * (long long)q + k];
                lo[k % 3] = fminf(lo[k % 3], v);
                hi[k % 3] = fmaxf(hi[k % 3], v);
            }
        for (int c = 0; c < 3; c++) {
            box[6 * f + c] = lo[c];
            box[6 * f + 3 + c] = hi[c];
        }
    }
}

void scene_face_tv(const SceneDev& s, hipStream_t st) {
    hipLaunchKernelGGL(k_face_tv, dim3(grid_for(s.T)), dim3(256), 0, st, s.T, s.face_tris, s.tris, s.verts,
                       s.face_tv);
    hipLaunchKernelGGL(k_face_box, dim3(grid_for(s.F)), dim3(256), 0, st, s.F, s.face_off, s.face_tv, s.face_box);
}

__global__ void k_tri_boxes(const int* list, int n, const int* tris, const float* verts, float* box) {
    GRID_STRIDE(k, (long long)n) {
        int t = list[k];
        const float* a = verts + 3 * tris[3 * t];
        const float* b = verts + 3 * tris[3 * t + 1];
        const float* c = verts + 3 * tris[3 * t + 2];
        for (int i = 0; i < 3; i++) {
            box[6 * k + i] = fminf(a[i], fminf(b[i], c[i]));
            box[6 * k + 3 + i] = fmaxf(a[i], fmaxf(b[i], c[i]));
        }
    }
}

void tri_boxes(const SceneDev& s, const int* list, int n, float* box6, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_tri_boxes, dim3(grid_for(n)), dim3(256), 0, st, list, n, s.tris, s.verts, box6);
}

__global__ void k_tri_prims(const int* list, const uint32_t* perm, int n, const int* tris, const int* tri_face,
                            const float* verts, TriP* prims) {
    GRID_STRIDE(sl, (long long)n) {
        int t = list[perm[sl]];
        const float* a = verts + 3 * tris[3 * t];
        const float* b = verts + 3 * tris[3 * t + 1];
        const float* c = verts + 3 * tris[3 * t + 2];
        TriP p;
        p.v0 = make_float4(a[0], a[1], a[2], __int_as_float(t));
        p.v1 = make_float4(b[0], b[1], b[2], __int_as_float(tri_face[t]));
        p.v2 = make_float4(c[0], c[1], c[2], 0.0f);
        prims[sl] = p;
    }
}

void tri_prims(const SceneDev& s, const int* list, const Tree& tree, TriP* prims, hipStream_t st) {
    if (tree.n > 0)
        hipLaunchKernelGGL(k_tri_prims, dim3(grid_for(tree.n)), dim3(256), 0, st, list, tree.perm, tree.n, s.tris,
                           s.tri_face, s.verts, prims);
}

__global__ void k_edge_static(int E, const int* rows, const int* face_dyn, uint32_t* is_static) {
    GRID_STRIDE(e, (long long)E) is_static[e] = face_dyn[rows[6 * e + 2]] < 0 ? 1u : 0u;
}

int edge_partition(SceneDev& s, uint32_t* scratch, int* count_dev, hipStream_t st) {
    s.E_s = 0;
    s.E_dyn = 0;
    if (s.E <= 0) return 0;
    uint32_t* flag = scratch;
    uint32_t* pos = flag + s.E;
    uint32_t* stemp = pos + s.E + 16;
    hipLaunchKernelGGL(k_edge_static, dim3(grid_for(s.E)), dim3(256), 0, st, s.E, s.edge_i, s.face_dyn, flag);
    exclusive_scan(flag, pos, s.E, stemp, (uint32_t*)count_dev, st);
    hipLaunchKernelGGL(k_partition, dim3(grid_for(s.E)), dim3(256), 0, st, s.E, flag, pos, s.edges_static,
                       s.edges_dynamic);
    int n = 0;
    hipError_t err = hipMemcpyAsync(&n, count_dev, sizeof(int), hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (err != hipSuccess) return -1;
    s.E_s = n;
    s.E_dyn = s.E - n;
    return n;
}

__global__ void k_edge_boxes(int n, const int* list, const int* rows, const float* verts, float* box) {
    GRID_STRIDE(i, (long long)n) {
        const int e = list[i];
        const float* a = verts + 3 * rows[6 * e];
        const float* b = verts + 3 * rows[6 * e + 1];
        for (int k = 0; k < 3; k++) {
            box[6 * i + k] = fminf(a[k], b[k]);
            box[6 * i + 3 + k] = fmaxf(a[k], b[k]);
        }
    }
}

void edge_boxes(const SceneDev& s, const int* list, int n, float* box6, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_edge_boxes, dim3(grid_for(n)), dim3(256), 0, st, n, list, s.edge_i, s.verts, box6);
}

__global__ void k_edge_prims(const int* list, const uint32_t* perm, int n, const int* rows, const float* verts,
                             float4* prims) {
    GRID_STRIDE(sl, (long long)n) {
        const int e = list[perm[sl]];
        const float* a = verts + 3 * rows[6 * e];
        const float* b = verts + 3 * rows[6 * e + 1];
        prims[2 * sl] = make_float4(a[0], a[1], a[2], __int_as_float(e));
        prims[2 * sl + 1] = make_float4(b[0], b[1], b[2], 0.0f);
    }
}

void edge_prims(const SceneDev& s, const int* list, const Tree& tree, float4* prims, hipStream_t st) {
    if (tree.n > 0)
        hipLaunchKernelGGL(k_edge_prims, dim3(grid_for(tree.n)), dim3(256), 0, st, list, tree.perm, tree.n, s.edge_i,
                           s.verts, prims);
}

__global__ void k_rx_boxes(const double* rx, int n, float* box) {
    GRID_STRIDE(i, (long long)n) {
        for (int c = 0; c < 3; c++) {
            float v = (float)rx[3 * i + c];
            box[6 * i + c] = v;
            box[6 * i + 3 + c] = v;
        }
    }
}

void rx_boxes(const double* rx_pos, int n_rx, float* box6, hipStream_t st) {
    if (n_rx > 0) hipLaunchKernelGGL(k_rx_boxes, dim3(grid_for(n_rx)), dim3(256), 0, st, rx_pos, n_rx, box6);
}

__global__ void k_rx_prims(const double* rx, const uint32_t* perm, int n, float4* prims) {
    GRID_STRIDE(sl, (long long)n) {
        int r = (int)perm[sl];
        prims[sl] = make_float4((float)rx[3 * r], (float)rx[3 * r + 1], (float)rx[3 * r + 2], __int_as_float(r));
    }
}

void rx_prims(const double* rx_pos, const Tree& tree, float4* prims, hipStream_t st) {
    if (tree.n > 0)
        hipLaunchKernelGGL(k_rx_prims, dim3(grid_for(tree.n)), dim3(256), 0, st, rx_pos, tree.perm, tree.n, prims);
}

}  // namespace emrt
