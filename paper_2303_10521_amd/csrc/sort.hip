// sort.hip -- device-wide exclusive scan and stable LSD radix sort of
// (u64 key, u32 value) pairs, written for wave64: digits are ranked inside a
// wave with eight ballots (lanes with equal digits), across the waves of a
// block through LDS, and across blocks through a scanned digit-major
// histogram.  Element counts may live in device memory so a frame needs no
// host round trip; `cap` bounds the launch.
#include "emrt_dev.h"
#include "emrt_launch.h"

namespace emrt {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 16;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;  // 4096
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;  // 2048

__device__ __forceinline__ long long dev_count(const long long* n_dev, long long cap) {
    if (!n_dev) return cap;
    long long n = *n_dev;
    return n < cap ? n : cap;
}

// ---------------------------------------------------------------- scan ----
// block-level exclusive scan of 256 values (returns the block total)
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
    int t = threadIdx.x;
    int lane = t & 63, w = t >> 6;
    // inclusive scan within the wave
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    uint32_t off = 0;
    for (int i = 0; i < w; i++) off += sh[i];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return off + x - v;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const uint32_t* in, long long n, uint32_t* sums) {
    __shared__ uint32_t sh[4];
    long long base = (long long)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; i++) {
        long long k = base + (long long)threadIdx.x * SCAN_ITEMS + i;
        if (k < n) s += in[k];
    }
    uint32_t total;
    block_excl_scan(s, sh, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// single block: exclusive scan of the block sums (any length, looped)
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_sums(uint32_t* sums, int nb, uint32_t* grand) {
    __shared__ uint32_t sh[4];
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += SCAN_THREADS) {
        int k = base + (int)threadIdx.x;
        uint32_t v = k < nb ? sums[k] : 0;
        uint32_t total;
        uint32_t ex = block_excl_scan(v, sh, total);
        if (k < nb) sums[k] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0 && grand) *grand = carry;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_apply(const uint32_t* in, uint32_t* out, long long n,
                                                            const uint32_t* sums) {
    __shared__ uint32_t sh[4];
    long long base = (long long)blockIdx.x * SCAN_TILE;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; i++) {
        long long k = base + (long long)threadIdx.x * SCAN_ITEMS + i;
        v[i] = k < n ? in[k] : 0;
        s += v[i];
    }
    uint32_t total;
    uint32_t ex = block_excl_scan(s, sh, total) + sums[blockIdx.x];
    for (int i = 0; i < SCAN_ITEMS; i++) {
        long long k = base + (long long)threadIdx.x * SCAN_ITEMS + i;
        if (k < n) out[k] = ex;
        ex += v[i];
    }
}

// single block over a short array: tile by tile with a running carry, so a
// scan of up to kScanSmall values is one launch instead of three
constexpr long long kScanSmall = 16LL * SCAN_TILE;
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_small(const uint32_t* in, uint32_t* out, long long n,
                                                            uint32_t* grand) {
    __shared__ uint32_t sh[4];
    uint32_t carry = 0;
    for (long long base = 0; base < n; base += SCAN_TILE) {
        uint32_t v[SCAN_ITEMS];
        uint32_t s = 0;
        for (int i = 0; i < SCAN_ITEMS; i++) {
            long long k = base + (long long)threadIdx.x * SCAN_ITEMS + i;
            v[i] = k < n ? in[k] : 0;
            s += v[i];
        }
        uint32_t total;
        uint32_t ex = block_excl_scan(s, sh, total) + carry;
        for (int i = 0; i < SCAN_ITEMS; i++) {
            long long k = base + (long long)threadIdx.x * SCAN_ITEMS + i;
            if (k < n) out[k] = ex;
            ex += v[i];
        }
        carry += total;
    }
    if (threadIdx.x == 0 && grand) *grand = carry;
}

size_t scan_temp_bytes(long long n) { return sizeof(uint32_t) * (size_t)((n + SCAN_TILE - 1) / SCAN_TILE + 1); }

void exclusive_scan(const uint32_t* in, uint32_t* out, long long n, uint32_t* temp, uint32_t* grand,
                    hipStream_t st) {
    int nb = (int)((n + SCAN_TILE - 1) / SCAN_TILE);
    if (nb == 0) {
        if (grand) hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, st, temp, 0, grand);
        return;
    }
    if (n <= kScanSmall) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(SCAN_THREADS), 0, st, in, out, n, grand);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(SCAN_THREADS), 0, st, in, n, temp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_THREADS), 0, st, temp, nb, grand);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(SCAN_THREADS), 0, st, in, out, n, temp);
}

// The same scan over the first min(*n_dev + add, cap) values, a count that
// lives in device memory: blocks past it return at once (their outputs are
// left unwritten) and the block sums are scanned up to it.
__device__ __forceinline__ long long live_count(const unsigned long long* n_dev, long long add, long long cap) {
    long long n = (long long)*n_dev + add;
    return n < cap ? n : cap;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce_dev(const uint32_t* in, const unsigned long long* n_dev,
                                                                 long long add, long long cap, uint32_t* sums) {
    __shared__ uint32_t sh[4];
    const long long n = live_count(n_dev, add, cap);
    long long base = (long long)blockIdx.x * SCAN_TILE;
    if (base >= n) return;
    uint32_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; i++) {
        long long k = base + (long long)threadIdx.x * SCAN_ITEMS + i;
        if (k < n) s += in[k];
    }
    uint32_t total;
    block_excl_scan(s, sh, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_sums_dev(uint32_t* sums, const unsigned long long* n_dev,
                                                               long long add, long long cap, uint32_t* grand) {
    __shared__ uint32_t sh[4];
    const long long n = live_count(n_dev, add, cap);
    const int nb = (int)((n + SCAN_TILE - 1) / SCAN_TILE);
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += SCAN_THREADS) {
        int k = base + (int)threadIdx.x;
        uint32_t v = k < nb ? sums[k] : 0;
        uint32_t total;
        uint32_t ex = block_excl_scan(v, sh, total);
        if (k < nb) sums[k] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0 && grand) *grand = carry;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_apply_dev(const uint32_t* in, uint32_t* out,
                                                                const unsigned long long* n_dev, long long add,
                                                                long long cap, const uint32_t* sums) {
    __shared__ uint32_t sh[4];
    const long long n = live_count(n_dev, add, cap);
    long long base = (long long)blockIdx.x * SCAN_TILE;
    if (base >= n) return;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
    for (int i = 0; i < SCAN_ITEMS; i++) {
        long long k = base + (long long)threadIdx.x * SCAN_ITEMS + i;
        v[i] = k < n ? in[k] : 0;
        s += v[i];
    }
    uint32_t total;
    uint32_t ex = block_excl_scan(s, sh, total) + sums[blockIdx.x];
    for (int i = 0; i < SCAN_ITEMS; i++) {
        long long k = base + (long long)threadIdx.x * SCAN_ITEMS + i;
        if (k < n) out[k] = ex;
        ex += v[i];
    }
}

void exclusive_scan_dev(const uint32_t* in, uint32_t* out, const unsigned long long* n_dev, long long add,
                        long long cap, uint32_t* temp, uint32_t* grand, hipStream_t st) {
    int nb = (int)((cap + SCAN_TILE - 1) / SCAN_TILE);
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_scan_reduce_dev, dim3(nb), dim3(SCAN_THREADS), 0, st, in, n_dev, add, cap, temp);
    hipLaunchKernelGGL(k_scan_sums_dev, dim3(1), dim3(SCAN_THREADS), 0, st, temp, n_dev, add, cap, grand);
    hipLaunchKernelGGL(k_scan_apply_dev, dim3(nb), dim3(SCAN_THREADS), 0, st, in, out, n_dev, add, cap, temp);
}

// ---------------------------------------------------------- radix sort ----
__global__ void __launch_bounds__(SORT_THREADS) k_radix_hist(const unsigned long long* keys, const long long* n_dev,
                                                            long long cap, int shift, int nblocks, uint32_t* hist) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    long long n = dev_count(n_dev, cap);
    long long base = (long long)blockIdx.x * SORT_TILE;
    for (int i = 0; i < SORT_ITEMS; i++) {
        long long k = base + (long long)i * SORT_THREADS + threadIdx.x;
        if (k < n) atomicAdd(&cnt[(uint32_t)(keys[k] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(long long)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(SORT_THREADS) k_radix_scatter(const unsigned long long* kin, const uint32_t* vin,
                                                               unsigned long long* kout, uint32_t* vout,
                                                               const long long* n_dev, long long cap, int shift,
                                                               int nblocks, const uint32_t* offs) {
    __shared__ uint32_t run[256];      // items of each digit already placed by this block
    __shared__ uint32_t wcnt[4][256];  // per-wave digit counts of the current round
    __shared__ uint32_t base_off[256];
    int t = threadIdx.x, lane = t & 63, w = t >> 6;
    run[t] = 0;
    for (int q = 0; q < 4; q++) wcnt[q][t] = 0;
    base_off[t] = offs[(long long)t * nblocks + blockIdx.x];
    __syncthreads();
    long long n = dev_count(n_dev, cap);
    long long base = (long long)blockIdx.x * SORT_TILE;
    if (base >= n) return;
    for (int i = 0; i < SORT_ITEMS; i++) {
        long long k = base + (long long)i * SORT_THREADS + t;
        bool ok = k < n;
        unsigned long long key = ok ? kin[k] : 0ULL;
        uint32_t val = ok ? vin[k] : 0u;
        uint32_t dg = ok ? (uint32_t)(key >> shift) & 255u : 256u;
        // lanes of this wave holding the same digit
        uint64_t peers = ballot64(ok);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            uint64_t m = ballot64((dg >> b) & 1u);
            peers &= ((dg >> b) & 1u) ? m : ~m;
        }
        int rank = prefix_below(peers);
        int leader = __ffsll((long long)peers) - 1;
        if (ok && lane == leader) wcnt[w][dg] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (ok) {
            uint32_t before = run[dg];
            for (int q = 0; q < w; q++) before += wcnt[q][dg];
            uint32_t dst = base_off[dg] + before + (uint32_t)rank;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
        wcnt[0][t] = 0; wcnt[1][t] = 0; wcnt[2][t] = 0; wcnt[3][t] = 0;
        __syncthreads();
    }
}

size_t radix_temp_bytes(long long cap) {
    long long nb = (cap + SORT_TILE - 1) / SORT_TILE;
    if (nb < 1) nb = 1;
    size_t h = sizeof(uint32_t) * 256 * (size_t)nb;
    return 2 * h + scan_temp_bytes(256 * nb) + 256;
}

// Sort `cap`-bounded pairs in (k0, v0) by key bits [0, nbits); k1/v1 are
// ping-pong buffers of the same size.  Returns 0 when the result is in k0/v0,
// 1 when it is in k1/v1.
int radix_sort(unsigned long long* k0, uint32_t* v0, unsigned long long* k1, uint32_t* v1, const long long* n_dev,
               long long cap, int nbits, void* temp, hipStream_t st) {
    if (cap <= 0) return 0;
    int nb = (int)((cap + SORT_TILE - 1) / SORT_TILE);
    uint32_t* hist = (uint32_t*)temp;
    uint32_t* offs = hist + 256 * (size_t)nb;
    uint32_t* stmp = offs + 256 * (size_t)nb;
    int passes = (nbits + 7) / 8;
    unsigned long long *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    for (int p = 0; p < passes; p++) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(SORT_THREADS), 0, st, ki, n_dev, cap, shift, nb, hist);
        exclusive_scan(hist, offs, 256LL * nb, stmp, nullptr, st);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(SORT_THREADS), 0, st, ki, vi, ko, vo, n_dev, cap, shift, nb,
                           offs);
        unsigned long long* tk = ki; ki = ko; ko = tk;
        uint32_t* tv = vi; vi = vo; vo = tv;
    }
    return (passes & 1) ? 1 : 0;
}

// ------------------------------------------------------------- fills ----
__global__ void k_fill_u32(uint32_t* p, uint32_t v, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long s = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += s) p[i] = v;
}
__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long s = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += s) p[i] = v;
}
__global__ void k_iota(uint32_t* p, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long s = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += s) p[i] = (uint32_t)i;
}

static int fill_grid(long long n) {
    long long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    return (int)(b < 1 ? 1 : b);
}

void fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(256), 0, st, p, v, n);
}
void fill_u64(unsigned long long* p, unsigned long long v, long long n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(n)), dim3(256), 0, st, p, v, n);
}
void iota_u32(uint32_t* p, long long n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_iota, dim3(fill_grid(n)), dim3(256), 0, st, p, n);
}

}  // namespace emrt
