// adjoint.hip -- gradients of a loss of the per-link channels with respect to
// the material permittivities, the transmitter positions and the dipole
// orientation, with the path topology of the last step held fixed.
//
// The paper computes channels only; the gradients are an extension.  With
// H_{f,l} = sum of the path amplitudes a of link l at carrier f and a real
// loss L(H, P_coh), the caller supplies G_H = dL/dRe H + j dL/dIm H and
// G_P = dL/dP_coh; with P_coh = P_tx |H|^2 the effective cotangent of H is
//   g = G_H + 2 P_tx G_P H,
// and for a real parameter x, dL/dx = sum Re(conj(g) da/dx); for a complex
// permittivity eps (a is holomorphic in eps), dL/dRe eps + j dL/dIm eps =
// sum g conj(da/deps).
//
// Work is spread over (valid path, derivative) items, so the GPU holds many
// times as many threads as valid paths:
//   * dual items rebuild the path's interaction points from the transmitter
//     position in forward-mode dual numbers (image method / Keller point,
//     fields.h) and evaluate the field in the same numbers, which gives
//     da/d(tx, theta, phi), one tangent direction per item;
//   * permittivity item md = 1..5 evaluates the field with interaction md's reflection
//     coefficients replaced by their eps-derivatives, which gives da/deps of
//     its material (a diffraction has two: its wedge faces; a path with one
//     reflection and one diffraction has three).
// Each item writes its path's partial sums (over carriers); then one thread
// per (row, link) adds the link's partials in key order into rows
// [5 + 2 M][n_links],
// and one block per output scalar sums the rows in a fixed order, so the
// result is bit-for-bit repeatable.
#include "emrt_dev.h"
#include "emrt_launch.h"
#include "fields.h"

namespace emrt {

// number of permittivity derivatives of a path (one per interaction)
__device__ __forceinline__ int n_modes(int type, int order) {
    return type == KT_SPEC ? order : (type == KT_DIFF ? 2 : (type >= KT_RD ? 3 : 0));
}

// material of interaction md (1-based) of a path
__device__ __forceinline__ int mode_material(const SceneDev& S, const KeyRec& key, int type, int md) {
    if (type == KT_SPEC) return S.face_material[key.ids[md - 1]];
    if (md == 3) return S.face_material[type == KT_RD ? key.ids[0] : key.ids[1]];
    return S.face_material[S.edge_i[6 * (long long)(type == KT_RD ? key.ids[1] : key.ids[0]) + (md == 1 ? 2 : 3)]];
}

// the link's effective cotangents of H, one per carrier
__device__ __forceinline__ void link_cotangent(const AdjArgs& a, long long l, cd* g) {
    const long long nl = a.n_links;
    for (int f = 0; f < a.fc.nf; f++) {
        const long long i = (long long)f * nl + l;
        g[f] = a.dL_dH ? C(a.dL_dH[2 * i], a.dL_dH[2 * i + 1]) : C(0.0);
        if (a.dL_dP) {
            const double* h = a.chan + 8 * i;
            g[f] = g[f] + C(h[0], h[1]) * (2.0 * a.p_tx * a.dL_dP[i]);
        }
    }
}

// Tangent directions per dual item: one (five light items per path) keeps
// the dual numbers in registers; all five in one item would need about five
// times the registers and spill.
constexpr int kAdjTan = 1;
constexpr int kAdjDual = kTan / kAdjTan;  // dual items per path
constexpr int kAdjEps = 5;                // permittivity items per path (the most interactions)

// KIND 0: every path type; 4: all but one reflection with one diffraction
// (the configurations that cannot produce them compile without that code).
template <int KIND>
__global__ void __launch_bounds__(128) k_adj_dual(AdjArgs a) {
    using DV = DNT<kAdjTan>;
    const SceneDev& S = a.s;
    long long n = (long long)*a.vp.count;
    if (n > a.vp.cap) n = a.vp.cap;
    for (long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x; it < n * kAdjDual;
         it += (long long)gridDim.x * blockDim.x) {
        const long long q = it / kAdjDual;
        const int t0 = (int)(it - q * kAdjDual) * kAdjTan;  // first tangent direction of this item
        const KeyRec key = a.vp.key[q];
        cd g[EMRT_NF];
        link_cotangent(a, (long long)key.tx * a.n_rx + key.rx, g);
        const double* tp = a.tx_pos + 3 * key.tx;
        const dv3 rx = ldd3(a.rx_pos + 3 * key.rx);
        V3<DV> s = v3<DV>(dn_seed<kAdjTan>(tp[0], 0, t0), dn_seed<kAdjTan>(tp[1], 1, t0),
                          dn_seed<kAdjTan>(tp[2], 2, t0));
        DV th = dn_seed<kAdjTan>(a.tx_orient[2 * key.tx], 3, t0);
        DV ph = dn_seed<kAdjTan>(a.tx_orient[2 * key.tx + 1], 4, t0);
        PathGeo<DV> gd;
        path_points<DV, KIND>(S, key, s, rx, gd);
        V3<DV> kk[EMRT_KMAX + 1];
        DV L;
        Cx<DV> amp[EMRT_NF];
        path_field<DV, KIND>(S, a.fc, key, gd, th, ph, 0, kk, L, amp);
        double acc[kAdjTan];
#pragma unroll
        for (int k = 0; k < kAdjTan; k++) acc[k] = 0.0;
        for (int f = 0; f < a.fc.nf; f++) {
#pragma unroll
            for (int k = 0; k < kAdjTan; k++) acc[k] += g[f].re * amp[f].re.d[k] + g[f].im * amp[f].im.d[k];
        }
#pragma unroll
        for (int k = 0; k < kAdjTan; k++) a.path_tan[kTan * q + t0 + k] = acc[k];
    }
}

// item (md, path): the field with interaction md's reflection coefficients
// replaced by their permittivity derivatives, the points at their values
// (the same image method / Keller point in double)
template <int KIND>
__global__ void __launch_bounds__(128) k_adj_eps(AdjArgs a) {
    const SceneDev& S = a.s;
    long long n = (long long)*a.vp.count;
    if (n > a.vp.cap) n = a.vp.cap;
    for (long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x; it < n * kAdjEps;
         it += (long long)gridDim.x * blockDim.x) {
        // interaction-major: the items of interactions a path lacks gather
        // in whole waves that end at once
        const int md = (int)(it / n) + 1;
        const long long q = it - (md - 1) * n;
        const KeyRec key = a.vp.key[q];
        const int type = key.to & 0xff, order = key.to >> 8;
        if (md > n_modes(type, order)) continue;  // the link sum reads only the items that exist
        double* out = a.path_eps + 2 * (kAdjEps * q + (md - 1));
        const int m = mode_material(S, key, type, md);
        if (m < 0 || m >= a.M) {
            out[0] = out[1] = 0.0;
            continue;
        }
        cd g[EMRT_NF];
        link_cotangent(a, (long long)key.tx * a.n_rx + key.rx, g);
        const double* tp = a.tx_pos + 3 * key.tx;
        PathGeo<double> gv;
        path_points<double, KIND>(S, key, v3c<double>(ldd3(tp)), ldd3(a.rx_pos + 3 * key.rx), gv);
        V3<double> kv[EMRT_KMAX + 1];
        double Lv;
        Cx<double> da[EMRT_NF];
        path_field<double, KIND>(S, a.fc, key, gv, a.tx_orient[2 * key.tx], a.tx_orient[2 * key.tx + 1], md, kv, Lv,
                                 da);
        double re = 0.0, im = 0.0;
        for (int f = 0; f < a.fc.nf; f++) {
            re += g[f].re * da[f].re + g[f].im * da[f].im;
            im += g[f].im * da[f].re - g[f].re * da[f].im;
        }
        out[0] = re;
        out[1] = im;
    }
}

// One thread per (row, link): the link's paths' partials of that row, in key
// order (rows 0..4: the real tangents; 5 + 2 m, 6 + 2 m: Re and Im of the
// permittivity of material m).  Consecutive threads take consecutive links
// of one row, so the row writes are coalesced.
__global__ void __launch_bounds__(256) k_adj_links(AdjArgs a) {
    const SceneDev& S = a.s;
    const long long nl = a.n_links;
    const long long n = (long long)(kTan + 2 * a.M) * nl;
    for (long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x; it < n;
         it += (long long)gridDim.x * blockDim.x) {
        const int row = (int)(it / nl);
        const long long l = it - (long long)row * nl;
        double acc = 0.0;
        const int p0 = a.start[l], p1 = a.end[l];
        if (p0 >= 0) {
            for (int p = p0; p < p1; p++) {
                const uint32_t q = a.order[p];
                if (row < kTan) {
                    acc += a.path_tan[kTan * (long long)q + row];
                    continue;
                }
                const int m = (row - kTan) >> 1, part = (row - kTan) & 1;
                const KeyRec key = a.vp.key[q];
                const int type = key.to & 0xff, order = key.to >> 8;
                const int nm = n_modes(type, order);
                for (int md = 1; md <= nm; md++)
                    if (mode_material(S, key, type, md) == m)
                        acc += a.path_eps[2 * (kAdjEps * (long long)q + (md - 1)) + part];
            }
        }
        a.rows[row * nl + l] = acc;
    }
}

// One block per output scalar: block b < 5 n_tx sums component b % 5 over
// the receivers of transmitter b / 5; the others sum a permittivity row over
// all links.  Strided partial sums, then a fixed LDS tree.
__global__ void __launch_bounds__(256) k_adj_reduce(const double* rows, long long n_links, int n_rx, int n_tx,
                                                    double* g_pos, double* g_ori, double* g_eps) {
    __shared__ double sh[256];
    const int b = blockIdx.x, t = threadIdx.x;
    const double* row;
    long long lo, n;
    double* out;
    if (b < 5 * n_tx) {
        int tx = b / 5, comp = b - 5 * tx;
        row = rows + (long long)comp * n_links;
        lo = (long long)tx * n_rx;
        n = n_rx;
        out = comp < 3 ? (g_pos ? g_pos + 3 * tx + comp : nullptr) : (g_ori ? g_ori + 2 * tx + comp - 3 : nullptr);
    } else {
        int r = b - 5 * n_tx;
        row = rows + (long long)(5 + r) * n_links;
        lo = 0;
        n = n_links;
        out = g_eps ? g_eps + r : nullptr;
    }
    double s = 0.0;
    for (long long i = t; i < n; i += 256) s += row[lo + i];
    sh[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0 && out) *out = sh[0];
}

void adjoint(const AdjArgs& a, int n_tx, int n_rx, double* g_pos, double* g_ori, double* g_eps, hipStream_t st) {
    // grids sized for the path capacity (they stride over the valid count)
    auto grid = [](long long items) {
        long long g = (items + 127) / 128;
        return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
    };
    if (a.combined) {
        hipLaunchKernelGGL(k_adj_dual<0>, dim3(grid(a.vp.cap * kAdjDual)), dim3(128), 0, st, a);
        hipLaunchKernelGGL(k_adj_eps<0>, dim3(grid(a.vp.cap * kAdjEps)), dim3(128), 0, st, a);
    } else {
        hipLaunchKernelGGL(k_adj_dual<4>, dim3(grid(a.vp.cap * kAdjDual)), dim3(128), 0, st, a);
        hipLaunchKernelGGL(k_adj_eps<4>, dim3(grid(a.vp.cap * kAdjEps)), dim3(128), 0, st, a);
    }
    long long gl = ((long long)(kTan + 2 * a.M) * a.n_links + 255) / 256;
    if (gl < 1) gl = 1;
    if (gl > 16384) gl = 16384;
    hipLaunchKernelGGL(k_adj_links, dim3((unsigned)gl), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_adj_reduce, dim3(5 * n_tx + 2 * a.M), dim3(256), 0, st, a.rows, a.n_links, n_rx, n_tx, g_pos,
                       g_ori, g_eps);
}

}  // namespace emrt
