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
// Per link (one thread, the link's paths in key order):
//   * the interaction points are rebuilt from the transmitter position with
//     forward-mode dual numbers (image method / Keller point, fields.h), and
//     the field evaluated in the same numbers gives da/d(tx, theta, phi);
//   * for every interaction, the field evaluated with that interaction's
//     reflection coefficients replaced by their eps-derivatives gives
//     da/deps of its material (a diffraction has two: its wedge faces; a
//     path with one reflection and one diffraction has three).
// The per-link partials go to rows [5 + 2 M][n_links]; a second kernel sums
// them in a fixed order (per transmitter over its receivers, per material
// over all links), so the result is deterministic.
#include "emrt_dev.h"
#include "emrt_launch.h"
#include "fields.h"

namespace emrt {

// KIND 0: every path type; 4: all but one reflection with one diffraction
// (the configurations that cannot produce them compile without that code).
template <int KIND>
__global__ void __launch_bounds__(128) k_adj_links(AdjArgs a) {
    const SceneDev& S = a.s;
    const long long nl = a.n_links;
    for (long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x; l < nl;
         l += (long long)gridDim.x * blockDim.x) {
        cd g[EMRT_NF];
        for (int f = 0; f < a.fc.nf; f++) {
            long long i = (long long)f * nl + l;
            g[f] = a.dL_dH ? C(a.dL_dH[2 * i], a.dL_dH[2 * i + 1]) : C(0.0);
            if (a.dL_dP) {
                const double* h = a.chan + 8 * i;
                g[f] = g[f] + C(h[0], h[1]) * (2.0 * a.p_tx * a.dL_dP[i]);
            }
        }
        for (int r = 0; r < 2 * a.M; r++) a.rows[(5 + r) * nl + l] = 0.0;
        double acc[kTan];
#pragma unroll
        for (int k = 0; k < kTan; k++) acc[k] = 0.0;
        int p0 = a.start[l], p1 = a.end[l];
        if (p0 >= 0) {
            for (int p = p0; p < p1; p++) {
                uint32_t q = a.order[p];
                KeyRec key = a.vp.key[q];
                const double* tp = a.tx_pos + 3 * key.tx;
                V3<DN> s = v3<DN>(dn_seed(tp[0], 0), dn_seed(tp[1], 1), dn_seed(tp[2], 2));
                DN th = dn_seed(a.tx_orient[2 * key.tx], 3), ph = dn_seed(a.tx_orient[2 * key.tx + 1], 4);
                dv3 rx = ldd3(a.rx_pos + 3 * key.rx);
                PathGeo<DN> gd;
                path_points<DN, KIND>(S, key, s, rx, gd);
                V3<DN> kk[EMRT_KMAX + 1];
                DN L;
                Cx<DN> amp[EMRT_NF];
                path_field<DN, KIND>(S, a.fc, key, gd, th, ph, 0, kk, L, amp);
                for (int f = 0; f < a.fc.nf; f++) {
#pragma unroll
                    for (int k = 0; k < kTan; k++) acc[k] += g[f].re * amp[f].re.d[k] + g[f].im * amp[f].im.d[k];
                }
                // permittivity: one evaluation per interaction
                int nmodes = gd.type == KT_SPEC ? gd.order : (gd.type == KT_DIFF ? 2 : (gd.type >= KT_RD ? 3 : 0));
                if (nmodes == 0) continue;
                PathGeo<double> gv;
#pragma unroll
                for (int i = 0; i < EMRT_KMAX + 2; i++) gv.P[i] = v3c<double>(val3(gd.P[i]));
                gv.Rx = v3c<double>(rx);
                gv.np = gd.np;
                gv.order = gd.order;
                gv.type = gd.type;
                for (int md = 1; md <= nmodes; md++) {
                    int m;
                    if (gd.type == KT_SPEC) m = S.face_material[key.ids[md - 1]];
                    else if (md == 3) m = S.face_material[gd.type == KT_RD ? key.ids[0] : key.ids[1]];
                    else m = S.face_material[S.edge_i[6 * (long long)(gd.type == KT_RD ? key.ids[1] : key.ids[0]) +
                                                      (md == 1 ? 2 : 3)]];
                    if (m < 0 || m >= a.M) continue;
                    V3<double> kv[EMRT_KMAX + 1];
                    double Lv;
                    Cx<double> da[EMRT_NF];
                    path_field<double, KIND>(S, a.fc, key, gv, th.v, ph.v, md, kv, Lv, da);
                    double re = 0.0, im = 0.0;
                    for (int f = 0; f < a.fc.nf; f++) {
                        re += g[f].re * da[f].re + g[f].im * da[f].im;
                        im += g[f].im * da[f].re - g[f].re * da[f].im;
                    }
                    a.rows[(5 + 2 * m) * nl + l] += re;
                    a.rows[(5 + 2 * m + 1) * nl + l] += im;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kTan; k++) a.rows[k * nl + l] = acc[k];
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
    long long g = (a.n_links + 127) / 128;
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    if (a.combined) hipLaunchKernelGGL(k_adj_links<0>, dim3((unsigned)g), dim3(128), 0, st, a);
    else hipLaunchKernelGGL(k_adj_links<4>, dim3((unsigned)g), dim3(128), 0, st, a);
    hipLaunchKernelGGL(k_adj_reduce, dim3(5 * n_tx + 2 * a.M), dim3(256), 0, st, a.rows, a.n_links, n_rx, n_tx, g_pos,
                       g_ori, g_eps);
}

}  // namespace emrt
