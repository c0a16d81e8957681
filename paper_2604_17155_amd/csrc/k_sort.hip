// Device-wide exclusive scan and stable LSD radix sort (digits of up to 8 bits).
//
// The sort orders the (view, Gaussian) items by depth and then the emitted
// (tile, item) pairs by tile.  Stability of every pass is what carries the
// depth order (and the index tie-break) into each tile's list.
#include <algorithm>

#include "gsc_internal.h"

namespace gsc {

namespace {
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;  // 2048

constexpr int kRsThreads = 512;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;  // 8192: runs of ~32 keys per digit
constexpr int kRsWaves = kRsThreads / 64;

__device__ inline uint32_t wave_inclusive_scan(uint32_t v) {
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive scan over the NT threads of a block; returns the block total in *total.
template <int NT = kScanThreads>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_inclusive_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, all = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) {
        uint32_t s = wsum[k];
        if (k < w) off += s;
        all += s;
    }
    *total = all;
    __syncthreads();
    return off + inc - v;
}
// The kScanItems = 8 consecutive elements at base: two 16-byte loads when
// they all lie below n and the array is 16-byte aligned, else one guarded
// load each (zero past the end).
__device__ inline void scan_load8(const uint32_t* in, uint64_t base, uint32_t n, uint32_t* x) {
    if (base + kScanItems <= n && (reinterpret_cast<uintptr_t>(in) & 15u) == 0) {
        const uint4 a = *reinterpret_cast<const uint4*>(in + base);
        const uint4 b = *reinterpret_cast<const uint4*>(in + base + 4);
        x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
        x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) x[j] = base + j < n ? in[base + j] : 0u;
    }
}
}  // namespace

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                              uint32_t n, uint32_t* __restrict__ bsums) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    uint64_t base = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanItems;
    uint32_t x[kScanItems];
    scan_load8(in, base, n, x);
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) s += x[j];
    uint32_t tot;
    block_exclusive_scan(s, wsum, &tot);
    if (threadIdx.x == 0) bsums[blockIdx.x] = tot;
}

// Down-sweep of one 2048-element block.  The block's offset is bsums[b] when
// the block sums have been scanned already; with `raw` they have not, and the
// block adds up bsums[0 .. b) itself (a few KB read from L2 for up to 2048
// blocks, in place of a launch that scans them).
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* in, uint32_t* out,
                                                            uint32_t n, const uint32_t* bsums,
                                                            uint32_t* total, int raw) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    uint32_t off = 0u;
    if (bsums && raw) {
        uint32_t part = 0u;
        for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kScanThreads) part += bsums[i];
        block_exclusive_scan(part, wsum, &off);
    } else if (bsums) {
        off = bsums[blockIdx.x];
    }
    uint64_t base = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanItems;
    uint32_t x[kScanItems];
    scan_load8(in, base, n, x);
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) s += x[j];
    uint32_t tot;
    uint32_t pre = block_exclusive_scan(s, wsum, &tot);
    pre += off;
    if (base + kScanItems <= n && (reinterpret_cast<uintptr_t>(out) & 15u) == 0) {
        uint32_t y[kScanItems];
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            y[j] = pre;
            pre += x[j];
        }
        *reinterpret_cast<uint4*>(out + base) = make_uint4(y[0], y[1], y[2], y[3]);
        *reinterpret_cast<uint4*>(out + base + 4) = make_uint4(y[4], y[5], y[6], y[7]);
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            uint64_t idx = base + j;
            if (idx < n) out[idx] = pre;
            pre += x[j];
        }
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
}

size_t scan_scratch_words(uint64_t n) {
    size_t w = 0;
    while (n > (uint64_t)kScanBlock) {
        n = (n + kScanBlock - 1) / kScanBlock;
        w += (size_t)((n + 63) / 64) * 64;
    }
    return w + 64;
}

void launch_scan(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* total, uint32_t* scratch,
                 hipStream_t s) {
    if (n == 0) {
        if (total) launch_fill_u32(total, 0u, 1, s);
        return;
    }
    if (n <= (uint32_t)kScanBlock) {
        hipLaunchKernelGGL(k_scan_down, dim3(1), dim3(kScanThreads), 0, s, in, out, n,
                           (const uint32_t*)nullptr, total, 0);
        return;
    }
    uint32_t nb = (n + kScanBlock - 1) / kScanBlock;
    uint32_t* bs = scratch;
    uint32_t* rest = scratch + ((nb + 63) / 64) * 64;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, in, n, bs);
    const int raw = nb <= (uint32_t)kScanBlock ? 1 : 0;
    if (!raw) launch_scan(bs, bs, nb, nullptr, rest, s);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanThreads), 0, s, in, out, n,
                       (const uint32_t*)bs, total, raw);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t step = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += step) p[i] = v;
}

// Fill with a kernel rather than hipMemsetAsync so that the work stays
// ordinary kernel nodes if a caller captures the stream into a graph.
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
    if (n == 0) return;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
}

// ---- radix sort ----------------------------------------------------------

// Digit histogram of one 8192-key tile, written digit-major: hist[d * nblocks + b]
// for the digits d <= mask of the pass ((key >> shift) & mask).
// n_dev (optional): the live key count, read on the device and clamped to n;
// the grid is sized for n.
__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint32_t* __restrict__ keys, uint32_t n,
                                                        const uint32_t* __restrict__ n_dev,
                                                        int shift, uint32_t mask, uint32_t* __restrict__ hist,
                                                        uint32_t nblocks) {
    if (n_dev) n = min(n, *n_dev);
    // four counter sets per wave (lane % 4): keys that share a digit, as in
    // the last pass of a sort whose top digit takes few values, spread their
    // LDS atomics over four addresses, which the padded rows (264 words: a
    // shift of 8 banks from one set to the next) put in different banks
    constexpr int kSets = 4, kRow = 264;
    __shared__ uint32_t h[kRsWaves * kSets][kRow];
    const int w = (int)(threadIdx.x >> 6) * kSets + (int)(threadIdx.x & (kSets - 1));
    const uint64_t base = (uint64_t)blockIdx.x * kRsTile;
    // All sixteen loads of a thread are issued before the counters are
    // cleared (sixteen coalesced loads in flight per wave, not one); an index
    // past the end reads the last key and is not counted.
    uint32_t kk[kRsItems];
    if (base < n) {
#pragma unroll
        for (int it = 0; it < kRsItems; ++it)
            kk[it] = keys[min(base + (uint64_t)it * kRsThreads + threadIdx.x, (uint64_t)n - 1)];
    }
    for (int k = threadIdx.x; k < kRsWaves * kSets * kRow; k += kRsThreads) (&h[0][0])[k] = 0;
    __syncthreads();
    if (base < n) {
#pragma unroll
        for (int it = 0; it < kRsItems; ++it)
            if (base + (uint64_t)it * kRsThreads + threadIdx.x < n)
                atomicAdd(&h[w][(kk[it] >> shift) & mask], 1u);
    }
    __syncthreads();
    uint32_t d = threadIdx.x;
    if (d > mask) return;
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kRsWaves * kSets; ++k) sum += h[k][d];
    hist[(uint64_t)d * nblocks + blockIdx.x] = sum;
}

// Stable scatter of one 8192-key tile (512 threads, 74 KB of LDS: two blocks
// and sixteen waves per CU).  Each wave ranks its 1024 keys (16 rounds of 64)
// against per-wave digit counters in LDS, with no block barrier; the eight
// waves' counts then give every key its position in the tile sorted by digit
// (threads 0..255 own one digit each).  The tile is reordered through LDS and written out in
// digit order, so each digit's run of keys is stored contiguously at the
// tile's offset for that digit.
//
// ONE_SWEEP = false: the offsets come from the scanned digit-major histogram
// `offs` of a separate histogram pass.  ONE_SWEEP = true: a single kernel per
// pass (decoupled look-back).  Each block takes the next tile number from a
// ticket counter, so every lower tile belongs to a block that is already
// running.  Once ranked, it publishes its per-digit counts in `status`, then
// adds up its predecessors' (a tile that has published its inclusive prefix
// ends the walk) and publishes its own inclusive prefix; the digit's start
// comes from the global digit counts `gcount`.  A status word holds the
// value in bits 0..29, kStAgg once the tile's own count is there and kStInc
// once its inclusive prefix is.  Every wait is bounded: after kLookbackSpins
// polls a block gives up, sets *fault (a word of the sort's scratch, not
// reported further) and goes on, so no kernel can hang; its output is then
// wrong, but only a predecessor that never publishes could cause that, and
// the ticket order guarantees every predecessor is running.
constexpr uint32_t kStAgg = 1u << 30, kStInc = 1u << 31, kStVal = kStAgg - 1u;
constexpr uint32_t kLookbackSpins = 1u << 22;

template <bool ONE_SWEEP>
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint32_t* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ vals_in,
                                                           uint32_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ vals_out,
                                                           uint32_t n, const uint32_t* __restrict__ n_dev, int shift, uint32_t mask,
                                                           const uint32_t* __restrict__ offs,
                                                           uint32_t nblocks, uint32_t* status,
                                                           const uint32_t* __restrict__ gcount,
                                                           uint32_t* ticket, uint32_t* fault) {
    if (n_dev) n = min(n, *n_dev);
    __shared__ uint32_t wcnt[kRsWaves][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t wsum[kRsThreads / 64];
    __shared__ uint32_t skey[kRsTile];
    __shared__ uint32_t sval[kRsTile];
    __shared__ uint32_t stile;
    uint32_t tile = blockIdx.x;
    if constexpr (ONE_SWEEP) {
        if (threadIdx.x == 0) stile = atomicAdd(ticket, 1u);
        __syncthreads();
        tile = stile;
    }
    if ((uint64_t)tile * kRsTile >= n) return;  // whole block: no live keys (no live tile follows)
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k = lane; k < 256; k += 64) wcnt[w][k] = 0u;
    if (!ONE_SWEEP && threadIdx.x <= mask) gbase[threadIdx.x] = offs[(uint64_t)threadIdx.x * nblocks + tile];
    const uint64_t tile0 = (uint64_t)tile * kRsTile;
    const uint64_t base = tile0 + (uint64_t)w * (kRsTile / kRsWaves);
    uint32_t kk[kRsItems], vv[kRsItems], rk[kRsItems];
    // The wave's 32 loads are all issued before the ranking, whose wave
    // barriers would otherwise hold each round's loads until the round
    // before has been ranked; an index past the end reads the last pair.
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        const uint64_t idx = min(base + (uint64_t)it * 64 + lane, (uint64_t)n - 1);
        kk[it] = keys_in[idx];
        vv[it] = vals_in[idx];
    }
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        const uint64_t idx = base + (uint64_t)it * 64 + lane;
        const bool valid = idx < n;
        const uint32_t key = kk[it];
        const uint32_t d = (key >> shift) & mask;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = __ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t pre = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        const uint32_t c = wcnt[w][d];
        __builtin_amdgcn_wave_barrier();
        if (valid && pre == 0) wcnt[w][d] = c + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
        rk[it] = valid ? c + pre : 0xFFFFFFFFu;
    }
    __syncthreads();
    {
        // thread t owns digit t: prefix over the waves, then over the digits
        const uint32_t t = threadIdx.x;
        uint32_t run = 0;
        if (t < 256) {
#pragma unroll
            for (int k = 0; k < kRsWaves; ++k) {
                const uint32_t c = wcnt[k][t];
                wcnt[k][t] = run;
                run += c;
            }
        }
        uint32_t tot;
        const uint32_t ds = block_exclusive_scan<kRsThreads>(run, wsum, &tot);
        if (t < 256) dstart[t] = ds;
        if constexpr (ONE_SWEEP) {
            // the digit's first output position, over all tiles
            const uint32_t gc = t <= mask ? gcount[t] : 0u;
            const uint32_t gstart = block_exclusive_scan<kRsThreads>(gc, wsum, &tot);
            if (t <= mask) {
                uint32_t* st = status + (uint64_t)tile * 256u + t;
                uint32_t excl = 0u;
                if (tile == 0u) {
                    __hip_atomic_store(st, kStInc | run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    __hip_atomic_store(st, kStAgg | run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    uint64_t j = tile - 1u;
                    uint32_t spins = 0u;
                    while (true) {
                        const uint32_t v = __hip_atomic_load(status + j * 256u + t, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                        if (v & kStInc) {
                            excl += v & kStVal;
                            break;
                        }
                        if (v & kStAgg) {  // tile 0 publishes its prefix at once: j stays >= 0
                            excl += v & kStVal;
                            --j;
                            continue;
                        }
                        if (++spins > kLookbackSpins) {
                            atomicOr(fault, 1u);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                    __hip_atomic_store(st, kStInc | (excl + run), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                gbase[t] = gstart + excl;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        if (rk[it] != 0xFFFFFFFFu) {
            const uint32_t d = (kk[it] >> shift) & mask;
            const uint32_t lp = dstart[d] + wcnt[w][d] + rk[it];
            skey[lp] = kk[it];
            sval[lp] = vv[it];
        }
    }
    __syncthreads();
    const uint32_t cnt = (uint32_t)min((uint64_t)kRsTile, (uint64_t)n - tile0);
    for (uint32_t i = threadIdx.x; i < cnt; i += kRsThreads) {
        const uint32_t key = skey[i];
        const uint32_t d = (key >> shift) & mask;
        const uint32_t gp = gbase[d] + (i - dstart[d]);
        keys_out[gp] = key;
        vals_out[gp] = sval[i];
    }
}

// The digit counts of every pass of a one-sweep sort, over all keys:
// gcount[p * 256 + d].  A grid of up to 2048 blocks strides over the 8192-key
// tiles; four counter sets per pass (lane mod 4) in padded rows, as in
// k_rs_hist, and one global atomic per block and non-zero count.
struct RadixDigits {
    int passes;
    int shift[4];
    uint32_t mask[4];
};
constexpr uint32_t kOneSweepHead = 1088;  // words before the status rows: gcount (1024), tickets, fault

__global__ __launch_bounds__(kRsThreads) void k_rs_counts(const uint32_t* __restrict__ keys, uint32_t n,
                                                          const uint32_t* __restrict__ n_dev, RadixDigits dg,
                                                          uint32_t* __restrict__ gcount) {
    if (n_dev) n = min(n, *n_dev);
    constexpr int kSets = 4, kRow = 264;
    __shared__ uint32_t h[4][kSets][kRow];
    for (int k = threadIdx.x; k < 4 * kSets * kRow; k += kRsThreads) (&h[0][0][0])[k] = 0u;
    __syncthreads();
    const uint32_t set = threadIdx.x & (kSets - 1);
    for (uint64_t base = (uint64_t)blockIdx.x * kRsTile; base < n; base += (uint64_t)gridDim.x * kRsTile) {
        uint32_t kk[kRsItems];
#pragma unroll
        for (int it = 0; it < kRsItems; ++it)
            kk[it] = keys[min(base + (uint64_t)it * kRsThreads + threadIdx.x, (uint64_t)n - 1)];
#pragma unroll
        for (int it = 0; it < kRsItems; ++it) {
            if (base + (uint64_t)it * kRsThreads + threadIdx.x >= n) continue;
            for (int p = 0; p < dg.passes; ++p) atomicAdd(&h[p][set][(kk[it] >> dg.shift[p]) & dg.mask[p]], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < dg.passes * 256; i += kRsThreads) {
        const int p = i >> 8, d = i & 255;
        const uint32_t c = h[p][0][d] + h[p][1][d] + h[p][2][d] + h[p][3][d];
        if (c != 0u) atomicAdd(&gcount[i], c);
    }
}

size_t radix_scratch_words(uint32_t n) {
    uint64_t nb = (n + kRsTile - 1) / kRsTile;
    uint64_t h = 256 * (nb > 0 ? nb : 1);
    const size_t classic = (size_t)(((h + 63) / 64) * 64 + scan_scratch_words(h));
    const size_t one_sweep = kOneSweepHead + 4 * (size_t)h;  // up to four passes of status rows
    return std::max(classic, one_sweep);
}

__global__ void k_copy_pairs(const uint32_t* __restrict__ ka, const uint32_t* __restrict__ va,
                             uint32_t* __restrict__ kb, uint32_t* __restrict__ vb, uint32_t n,
                             const uint32_t* __restrict__ n_dev) {
    if (n_dev) n = min(n, *n_dev);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        kb[i] = ka[i];
        vb[i] = va[i];
    }
}

void radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, uint32_t n,
                int bits, uint32_t* scratch, hipStream_t s, const uint32_t* n_dev, bool* result_in_alt) {
    if (result_in_alt) *result_in_alt = false;
    if (n <= 1 || bits <= 0) return;
    uint32_t nb = (n + kRsTile - 1) / kRsTile;
    uint32_t* hist = scratch;
    uint32_t* sscr = scratch + ((256ull * nb + 63) / 64) * 64;
    // as many passes as 8-bit digits need, with the bits spread evenly over
    // them (19 bits: 7 + 6 + 6): narrower digits leave longer runs of equal
    // digits in each tile, so the scattered writes come in fuller lines
    const int passes = (bits + 7) / 8;
    RadixDigits dg{passes, {0, 0, 0, 0}, {0u, 0u, 0u, 0u}};
    for (int p = 0, sh = 0; p < passes; ++p) {
        const int width = bits / passes + (p < bits % passes ? 1 : 0);
        dg.shift[p] = sh;
        dg.mask[p] = (1u << width) - 1u;
        sh += width;
    }
    // One sweep per pass for large sorts (where the status words can hold
    // every count); the scratch then holds [global digit counts | tickets,
    // fault | status rows].  Below 2^25 keys the look-back's waits cost more
    // than the histogram pass and scan they save (a 2^24-key depth sort: 0.45
    // against 0.37 ms; a 10^8-key pair sort of two passes: 1.09 against 1.26).
    const bool one_sweep = n >= (1u << 25) && n < kStAgg;
    uint32_t* gcount = scratch;
    uint32_t* tickets = scratch + 1024;
    uint32_t* fault = scratch + 1024 + 4;
    uint32_t* status = scratch + kOneSweepHead;
    if (one_sweep) {
        launch_fill_u32(scratch, 0u, kOneSweepHead + (uint64_t)passes * 256u * nb, s);
        hipLaunchKernelGGL(k_rs_counts, dim3(std::min<uint32_t>(nb, 2048u)), dim3(kRsThreads), 0, s, keys, n,
                           n_dev, dg, gcount);
    }
    uint32_t *sk = keys, *sv = vals, *dk = keys_alt, *dv = vals_alt;
    for (int p = 0; p < passes; ++p) {
        const int shift = dg.shift[p];
        const uint32_t mask = dg.mask[p];
        if (one_sweep) {
            hipLaunchKernelGGL(k_rs_scatter<true>, dim3(nb), dim3(kRsThreads), 0, s, sk, sv, dk, dv, n, n_dev,
                               shift, mask, (const uint32_t*)nullptr, nb, status + (uint64_t)p * 256u * nb,
                               gcount + 256 * p, tickets + p, fault);
        } else {
            hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(kRsThreads), 0, s, sk, n, n_dev, shift, mask, hist, nb);
            launch_scan(hist, hist, (mask + 1u) * nb, nullptr, sscr, s);
            hipLaunchKernelGGL(k_rs_scatter<false>, dim3(nb), dim3(kRsThreads), 0, s, sk, sv, dk, dv, n, n_dev,
                               shift, mask, hist, nb, (uint32_t*)nullptr, (const uint32_t*)nullptr,
                               (uint32_t*)nullptr, (uint32_t*)nullptr);
        }
        uint32_t* t;
        t = sk; sk = dk; dk = t;
        t = sv; sv = dv; dv = t;
    }
    if (sk != keys && result_in_alt) {
        *result_in_alt = true;  // the caller takes the result from the alternate buffers
    } else if (sk != keys) {
        // odd pass count: copy back with a kernel (plain kernel nodes under graph capture)
        const uint32_t blocks = std::min<uint32_t>((n + 255) / 256, 8192u);
        hipLaunchKernelGGL(k_copy_pairs, dim3(blocks), dim3(256), 0, s, sk, sv, keys, vals, n, n_dev);
    }
}

__global__ void k_tile_work_keys(const uint2* __restrict__ ranges, uint32_t n_bins,
                                 uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_bins) return;
    const uint2 r = ranges[b];
    // the octave of the list length, longest first; index order within one
    // octave keeps neighbouring tiles of a view together (shared records in L2)
    keys[b] = 31u - (31u - __clz(r.y - r.x + 1u));
    vals[b] = b;
}

size_t tile_order_words(uint32_t n_bins) {
    return 4 * (size_t)n_bins + radix_scratch_words(n_bins);
}

const uint32_t* launch_tile_order(const uint2* ranges, uint32_t n_bins, uint32_t* work, hipStream_t s) {
    uint32_t *keys = work, *vals = work + n_bins, *keys_alt = work + 2 * (size_t)n_bins,
             *vals_alt = work + 3 * (size_t)n_bins;
    if (n_bins == 0) return vals;
    hipLaunchKernelGGL(k_tile_work_keys, dim3((n_bins + 255) / 256), dim3(256), 0, s, ranges, n_bins, keys, vals);
    radix_sort(keys, vals, keys_alt, vals_alt, n_bins, 5, work + 4 * (size_t)n_bins, s);
    return vals;
}

}  // namespace gsc
