// bh_sort.hip -- device-wide exclusive scan and stable LSD radix sort.
//
// The sort orders the particles' 63-bit keys for the tree build; the paper
// names sorting as the dominant cost of tree construction (Sec. 4.2) and
// uses a sample sort on its CPEs.  Here it is a least-significant-digit
// radix sort with 8-bit digits: per pass one histogram kernel, one scan of
// the (digit, block) counts and one scatter kernel whose ranks come from
// wave-level digit matching (eight ballots), so equal keys keep their input
// order (stable).  The scatter first orders its tile by digit in LDS and then
// writes each digit's run to consecutive addresses.
#include "bh_internal.hpp"

namespace {

constexpr int SCAN_BLOCKS = 256;
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 4;

constexpr int RS_THREADS = 256;              // 4 waves
constexpr int RS_WAVE_ITEMS = 8;             // rounds of 64 keys per wave
constexpr int RS_TILE = RS_THREADS * RS_WAVE_ITEMS;   // 2048 keys per block

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *wsum, uint32_t *total) {
    // 256 threads = 4 waves; wsum: 4 words of LDS
    uint32_t inc = wave_incl_scan(v);
    int w = threadIdx.x >> 6;
    if (__lane_id() == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_THREADS / 64; ++k) {
        uint32_t t = wsum[k];
        off += (k < w) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const uint32_t *in, const uint32_t *n_dev,
                                                             uint32_t n_host, uint32_t *part) {
    __shared__ uint32_t wsum[4];
    uint32_t n = n_dev ? *n_dev : n_host;
    uint32_t chunk = (n + SCAN_BLOCKS - 1) / SCAN_BLOCKS;
    uint32_t b0 = blockIdx.x * chunk;
    uint32_t b1 = min(n, b0 + chunk);
    uint32_t s = 0;
    for (uint32_t i = b0 + threadIdx.x; i < b1; i += SCAN_THREADS) s += in[i];
    s = wave_sum(s);
    if (__lane_id() == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_top(uint32_t *part, uint32_t *total) {
    __shared__ uint32_t wsum[4];
    uint32_t v = part[threadIdx.x];
    uint32_t tot;
    uint32_t ex = block_excl_scan(v, wsum, &tot);
    part[threadIdx.x] = ex;
    if (threadIdx.x == 0 && total) *total = tot;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down(const uint32_t *in, uint32_t *out,
                                                           const uint32_t *n_dev, uint32_t n_host,
                                                           const uint32_t *part) {
    __shared__ uint32_t wsum[4];
    uint32_t n = n_dev ? *n_dev : n_host;
    uint32_t chunk = (n + SCAN_BLOCKS - 1) / SCAN_BLOCKS;
    uint32_t b0 = blockIdx.x * chunk;
    uint32_t b1 = min(n, b0 + chunk);
    uint32_t carry = part[blockIdx.x];
    for (uint32_t t0 = b0; t0 < b1; t0 += SCAN_THREADS * SCAN_ITEMS) {
        uint32_t v[SCAN_ITEMS];
        uint32_t base = t0 + threadIdx.x * SCAN_ITEMS;
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            v[k] = (base + k < b1) ? in[base + k] : 0u;
            s += v[k];
        }
        uint32_t tot;
        uint32_t ex = block_excl_scan(s, wsum, &tot) + carry;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            if (base + k < b1) out[base + k] = ex;
            ex += v[k];
        }
        carry += tot;
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------- radix sort
// Digit of element i: 8 key bits at `shift`, or (SYS) 8 bits of the system
// index that owns input index val[i] (sys_off: n_sys+1 ascending offsets).
template <bool SYS>
__device__ __forceinline__ uint32_t rs_digit(const uint64_t *key, const uint32_t *val, uint32_t i, int shift,
                                             const uint32_t *sys_off, int n_sys) {
    if (!SYS) return (uint32_t)(key[i] >> shift) & 255u;
    uint32_t v = val[i];
    int lo = 0, hi = n_sys - 1;          // last s with sys_off[s] <= v
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (sys_off[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return ((uint32_t)lo >> shift) & 255u;
}

template <bool SYS>
__global__ void __launch_bounds__(RS_THREADS) k_radix_hist(const uint64_t *key, const uint32_t *val, uint32_t n,
                                                          int shift, uint32_t *hist, uint32_t nb,
                                                          const uint32_t *sys_off, int n_sys) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    uint32_t base = blockIdx.x * RS_TILE;
#pragma unroll 4
    for (int r = 0; r < RS_WAVE_ITEMS; ++r) {
        uint32_t i = base + r * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&cnt[rs_digit<SYS>(key, val, i, shift, sys_off, n_sys)], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

template <bool SYS>
__global__ void __launch_bounds__(RS_THREADS) k_radix_scatter(const uint64_t *key_in, const uint32_t *val_in,
                                                             uint64_t *key_out, uint32_t *val_out,
                                                             uint32_t n, int shift,
                                                             const uint32_t *hist_scan, uint32_t nb,
                                                             const uint32_t *sys_off, int n_sys) {
    __shared__ uint32_t run[4][256];
    __shared__ uint32_t loc[256];                // block-local start of each digit's run
    __shared__ uint32_t gbase[256];              // global start of this block's run of each digit
    __shared__ uint32_t wsum[4];
    __shared__ uint64_t skey[RS_TILE];           // the tile in (digit, input) order
    __shared__ uint32_t sval[RS_TILE];
    __shared__ uint8_t sdig[RS_TILE];
    const int w = threadIdx.x >> 6;
    const int lane = __lane_id();
#pragma unroll
    for (int k = 0; k < 4; ++k) run[k][threadIdx.x] = 0;
    __syncthreads();

    const uint32_t base = blockIdx.x * RS_TILE + w * (RS_WAVE_ITEMS * 64);
    uint32_t digit[RS_WAVE_ITEMS];
    uint32_t rank[RS_WAVE_ITEMS];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < RS_WAVE_ITEMS; ++r) {
        uint32_t i = base + r * 64 + lane;
        bool valid = i < n;
        uint32_t d = valid ? rs_digit<SYS>(key_in, val_in, i, shift, sys_off, n_sys) : 0u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t old = valid ? run[w][d] : 0u;
        __syncthreads();
        bool leader = valid && ((peers & lt) == 0);
        if (leader) run[w][d] = old + (uint32_t)__popcll(peers);
        __syncthreads();
        digit[r] = d;
        rank[r] = old + (uint32_t)__popcll(peers & lt);
    }
    // block-local start of each digit (scan over the digits), then of each
    // wave's share of it; the block's global start of each digit
    {
        const uint32_t t = threadIdx.x;
        const uint32_t c0 = run[0][t], c1 = run[1][t], c2 = run[2][t], c3 = run[3][t];
        uint32_t tot;
        const uint32_t ex = block_excl_scan(c0 + c1 + c2 + c3, wsum, &tot);
        loc[t] = ex;
        run[0][t] = ex;
        run[1][t] = ex + c0;
        run[2][t] = ex + c0 + c1;
        run[3][t] = ex + c0 + c1 + c2;
        gbase[t] = hist_scan[t * nb + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_WAVE_ITEMS; ++r) {
        const uint32_t i = base + r * 64 + lane;
        if (i < n) {
            const uint32_t lp = run[w][digit[r]] + rank[r];
            skey[lp] = key_in[i];
            sval[lp] = val_in[i];
            sdig[lp] = (uint8_t)digit[r];
        }
    }
    __syncthreads();
    // consecutive threads write consecutive slots of each digit's run
    const uint32_t t0 = blockIdx.x * RS_TILE;
    const uint32_t cnt = n - t0 < (uint32_t)RS_TILE ? n - t0 : (uint32_t)RS_TILE;
    for (uint32_t p = threadIdx.x; p < cnt; p += RS_THREADS) {
        const uint32_t d = sdig[p];
        const uint32_t pos = gbase[d] + (p - loc[d]);
        key_out[pos] = skey[p];
        val_out[pos] = sval[p];
    }
}

}  // namespace

namespace bhk {

void scan_u32(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint32_t n_host,
              uint32_t *total, uint32_t *tmp, hipStream_t s) {
    k_scan_reduce<<<SCAN_BLOCKS, SCAN_THREADS, 0, s>>>(in, n_dev, n_host, tmp);
    k_scan_top<<<1, SCAN_THREADS, 0, s>>>(tmp, total);
    k_scan_down<<<SCAN_BLOCKS, SCAN_THREADS, 0, s>>>(in, out, n_dev, n_host, tmp);
}

void fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
    if (n == 0) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_fill_u32<<<(unsigned)blocks, 256, 0, s>>>(p, v, n);
}

size_t radix_hist_words(uint32_t n) {
    size_t nb = (n + RS_TILE - 1) / RS_TILE;
    if (nb == 0) nb = 1;
    return nb * 256;
}

void radix_sort(uint64_t *key_a, uint32_t *val_a, uint64_t *key_b, uint32_t *val_b,
                uint32_t n, int lo_bit, int hi_bit, uint32_t *hist, uint32_t *tmp, hipStream_t s,
                const uint32_t *sys_off, int n_sys) {
    if (n == 0) return;
    uint32_t nb = (n + RS_TILE - 1) / RS_TILE;
    uint64_t *ki = key_a, *ko = key_b;
    uint32_t *vi = val_a, *vo = val_b;
    int passes = 0;
    auto pass = [&](bool sys, int sh) {
        if (sys) {
            k_radix_hist<true><<<nb, RS_THREADS, 0, s>>>(ki, vi, n, sh, hist, nb, sys_off, n_sys);
        } else {
            k_radix_hist<false><<<nb, RS_THREADS, 0, s>>>(ki, vi, n, sh, hist, nb, sys_off, n_sys);
        }
        scan_u32(hist, hist, nullptr, nb * 256, nullptr, tmp, s);
        if (sys) {
            k_radix_scatter<true><<<nb, RS_THREADS, 0, s>>>(ki, vi, ko, vo, n, sh, hist, nb, sys_off, n_sys);
        } else {
            k_radix_scatter<false><<<nb, RS_THREADS, 0, s>>>(ki, vi, ko, vo, n, sh, hist, nb, sys_off, n_sys);
        }
        uint64_t *kt = ki; ki = ko; ko = kt;
        uint32_t *vt = vi; vi = vo; vo = vt;
        ++passes;
    };
    for (int sh = lo_bit; sh < hi_bit; sh += 8) pass(false, sh);
    // systems are the most significant digit: a final stable pass per 8 bits of system index
    if (sys_off && n_sys > 1)
        for (int sh = 0; (n_sys - 1) >> sh; sh += 8) pass(true, sh);
    if (passes & 1) {
        (void)hipMemcpyAsync(key_a, ki, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
        (void)hipMemcpyAsync(val_a, vi, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    }
}

}  // namespace bhk
