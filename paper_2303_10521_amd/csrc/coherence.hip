// coherence.hip -- per-link coherence statistics over frames (Section III-B):
// the channel correlation of Eq (1), the coherence time of Eq (2) and the
// spatial-consistency triggers of the trajectory segmentation (Section
// III-A), which together tell the caller when to rediscover paths instead of
// revalidating the cache.
//
// Readings (the paper prints the formulas, not their estimators):
//   Eq (1): the normalised autocovariance of g = |H| at lags of k frames,
//     R(k) = (mean_{t>=k} g_t g_{t-k} - m^2) / (mean g_t^2 - m^2), m = mean g_t,
//     over all frames since the last reset (NaN while undefined);
//   Eq (2): T_c = sqrt(1/R^4 - 1) / (2 pi f_D theta^2), f_D = f_c |v| / c for
//     the link's relative velocity v = v_rx - v_tx, theta the acute angle
//     between the line of motion and the transmitter -> receiver direction,
//     +inf when f_D theta^2 = 0;
//   triggers: bit 0 the line-of-sight flag changed since the previous step,
//     bit 1 the set of first-order paths (one reflection or one diffraction)
//     changed (compared through an order-independent hash of the keys).
// Updated once per step, after the per-link sums; the frame count lives on
// the device so replayed graphs advance it too.
#include "emrt_dev.h"
#include "emrt_launch.h"

namespace emrt {

__device__ __forceinline__ uint64_t first_order_hash(const KeyRec& k) {
    return mix64(((uint64_t)(uint32_t)k.tx << 40) ^ ((uint64_t)(uint32_t)k.rx << 8) ^ (uint64_t)(k.to & 0xff) ^
                 ((uint64_t)(uint32_t)k.ids[0] << 20) ^ 0x5bd1e995ULL);
}

__global__ void __launch_bounds__(256) k_coh_update(CohState c, ValidPaths vp, const uint32_t* order, const int* start,
                                                    const int* end, const double* chan, long long n_links, int nf) {
    const unsigned long long t = *c.frames;
    const int* chan_i = (const int*)(chan + (long long)nf * n_links * 8);
    for (long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x; l < n_links;
         l += (long long)gridDim.x * blockDim.x) {
        uint32_t los = chan_i[2 * l + 1] ? 1u : 0u;
        uint64_t h = 0;
        int s = start[l], e = end[l];
        if (s >= 0)
            for (int p = s; p < e; p++) {
                KeyRec k = vp.key[order[p]];
                int type = k.to & 0xff, ord = k.to >> 8;
                if (ord == 1 && (type == KT_SPEC || type == KT_DIFF)) h += first_order_hash(k);
            }
        uint32_t trig = 0;
        if (t > 0) trig = (los != c.prev_los[l] ? 1u : 0u) | (h != c.prev_hash[l] ? 2u : 0u);
        c.trigger[l] = trig;
        c.prev_los[l] = los;
        c.prev_hash[l] = h;
        for (int f = 0; f < nf; f++) {
            long long i = (long long)f * n_links + l;
            double g = hypot(chan[8 * i], chan[8 * i + 1]);
            double* ring = c.ring + i * EMRT_CORR_LAGS;
            double* prod = c.prod + i * EMRT_CORR_LAGS;
#pragma unroll
            for (int k = 1; k <= EMRT_CORR_LAGS; k++)
                if (t >= (unsigned long long)k) prod[k - 1] += g * ring[(t - k) % EMRT_CORR_LAGS];
            c.s1[i] += g;
            c.s2[i] += g * g;
            ring[t % EMRT_CORR_LAGS] = g;
        }
    }
}

__global__ void k_coh_advance(unsigned long long* frames) { *frames += 1ULL; }

void coherence_update(const CohState& c, const ValidPaths& vp, const uint32_t* order, const int* start,
                      const int* end, const double* chan, long long n_links, int nf, hipStream_t st) {
    long long g = (n_links + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_coh_update, dim3((unsigned)g), dim3(256), 0, st, c, vp, order, start, end, chan, n_links,
                       nf);
    hipLaunchKernelGGL(k_coh_advance, dim3(1), dim3(1), 0, st, c.frames);
}

// Eq (2) and the Eq (1) estimates for every link and carrier; min_tc (the
// smallest finite T_c, as the bit pattern of a non-negative double, so an
// integer minimum orders it) and the number of triggered links.
__global__ void __launch_bounds__(256) k_coh_read(CohState c, CohRead r, long long n_links, int n_rx, int nf,
                                                  const double* tx_pos, const double* tx_vel, const double* rx_pos,
                                                  const double* rx_vel, FieldCtx fc) {
    const double n = (double)*c.frames;
    const double num = sqrt(1.0 / (r.R * r.R * r.R * r.R) - 1.0);
    for (long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x; l < n_links;
         l += (long long)gridDim.x * blockDim.x) {
        int tx = (int)(l / n_rx), rx = (int)(l - (long long)tx * n_rx);
        dv3 v = ldd3(rx_vel + 3 * rx) - ldd3(tx_vel + 3 * tx);
        dv3 d = ldd3(rx_pos + 3 * rx) - ldd3(tx_pos + 3 * tx);
        double vn = len(v), dn = len(d);
        double theta = 0.0;
        if (vn > 0.0 && dn > 0.0) theta = acos(fmin(1.0, fabs(dot(v, d)) / (vn * dn)));
        uint32_t trig = c.trigger[l];
        if (r.trigger) r.trigger[l] = trig;
        if (trig && r.n_triggered) atomicAdd(r.n_triggered, 1ULL);
        for (int f = 0; f < nf; f++) {
            long long i = (long long)f * n_links + l;
            double fd = fc.freq[f] * vn / kC0;
            double den = 2.0 * kPi * fd * theta * theta;
            double tc = den > 0.0 ? num / den : INFINITY;
            if (r.tc) r.tc[i] = tc;
            if (den > 0.0 && r.min_tc) atomicMin(r.min_tc, (unsigned long long)__double_as_longlong(tc));
            if (r.corr) {
                double m = c.s1[i] / n, var = c.s2[i] / n - m * m;
#pragma unroll
                for (int k = 1; k <= EMRT_CORR_LAGS; k++) {
                    double val = NAN;
                    if (n > (double)k && var != 0.0) val = (c.prod[i * EMRT_CORR_LAGS + k - 1] / (n - k) - m * m) / var;
                    r.corr[i * EMRT_CORR_LAGS + k - 1] = val;
                }
            }
        }
    }
}

void coherence_read(const CohState& c, const CohRead& r, long long n_links, int n_rx, int nf, const double* tx_pos,
                    const double* tx_vel, const double* rx_pos, const double* rx_vel, const FieldCtx& fc,
                    hipStream_t st) {
    long long g = (n_links + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_coh_read, dim3((unsigned)g), dim3(256), 0, st, c, r, n_links, n_rx, nf, tx_pos, tx_vel, rx_pos,
                       rx_vel, fc);
}

}  // namespace emrt
