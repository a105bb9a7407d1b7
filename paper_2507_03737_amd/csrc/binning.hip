// Tile binning: exclusive scan of per-record tile counts, (tile, record) pair emission,
// a stable LSD radix sort and per-tile ranges.
//
// Every Gaussian-view record is first sorted by its float32 camera depth (the paper
// composites "sorted by z_k", Sec. 3.2.1, Eq. 3); pairs are then emitted in that order
// and stably sorted by global tile id, so each tile's list comes out ordered by
// (depth, record index) without ever carrying depth bits in the large pair sort.  The
// pair count is only known on the device: all kernels after the scan read it from
// device memory and use fixed grids, so the whole sequence can be captured in a graph.
#include "gspm_common.h"

namespace gspm {

namespace {

// ------------------------------- scan --------------------------------------------------

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ inline uint32_t load_count(const uint32_t *counts, const uint32_t *idx, int64_t p, int flag) {
    if (flag == 2) {
        const uint32_t v = idx[p];
        const uint32_t c = v >> kPackShift;
        return c < kPackCountMax ? c : counts[v & kPackMask];
    }
    const uint32_t c = idx ? counts[idx[p]] : counts[p];
    return flag ? (c != 0u ? 1u : 0u) : c;
}

// Elements per block of the device-wide scans: a multiple of kScanItems, so that every
// thread's group of kScanItems consecutive words starts 32-byte aligned.
__device__ inline int64_t scan_chunk(int64_t n) {
    const int64_t c = (n + gridDim.x - 1) / gridDim.x;
    return (c + kScanItems - 1) / kScanItems * kScanItems;
}

__device__ inline int64_t scan_n(const uint32_t *n_dev, int64_t n_max) {
    if (!n_dev) return n_max;
    const int64_t n = (int64_t)*n_dev;
    return n < n_max ? n : n_max;
}

// Block-wide exclusive scan of one value per thread (NW waves); returns the prefix, *total
// the sum.
template <int NW = kScanBlock / kWave>
__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t *lds, uint32_t &total) {
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const uint32_t inc = wave_inclusive_scan(x);
    if (lane == kWave - 1) lds[wid] = inc;
    __syncthreads();
    uint32_t wave_base = 0, tot = 0;
    for (int k = 0; k < NW; ++k) {
        const uint32_t t = lds[k];
        if (k < wid) wave_base += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return wave_base + inc - x;
}

__global__ void __launch_bounds__(kScanBlock)
k_scan_reduce(const uint32_t *__restrict__ counts, const uint32_t *__restrict__ idx, const uint32_t *__restrict__ n_dev,
              int64_t n_max, int flag, uint32_t *__restrict__ part, uint32_t *__restrict__ gathered) {
    __shared__ uint32_t lds[kScanBlock / kWave];
    const int64_t n = scan_n(n_dev, n_max);
    const int64_t chunk = scan_chunk(n);
    const int64_t b0 = (int64_t)blockIdx.x * chunk < n ? (int64_t)blockIdx.x * chunk : n;
    const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
    uint32_t acc = 0;
    // kScanItems loads per thread in flight at once, each instruction over consecutive words.
    for (int64_t base = b0; base < b1; base += kScanTile) {
        uint32_t c[kScanItems];
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int64_t p = base + k * kScanBlock + threadIdx.x;
            c[k] = p < b1 ? load_count(counts, idx, p, flag) : 0u;
        }
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int64_t p = base + k * kScanBlock + threadIdx.x;
            if (gathered && p < b1) gathered[p] = c[k];
            acc += c[k];
        }
    }
    uint32_t tot;
    block_exclusive_scan(acc, lds, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// The sum of the block partials before this block, and in `all` the sum of every block's:
// each block adds them itself (at most kScanMaxBlocks words, all loads in flight at once),
// which spares a separate launch that would scan them.
__device__ inline uint32_t partial_prefix(const uint32_t *__restrict__ part, uint32_t *lds, uint32_t &all) {
    constexpr int kPer = kScanMaxBlocks / kScanBlock;
    uint32_t v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int b = (int)threadIdx.x + q * kScanBlock;
        v[q] = b < (int)gridDim.x ? part[b] : 0u;
    }
    uint32_t before = 0u, every = 0u;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        every += v[q];
        before += (int)threadIdx.x + q * kScanBlock < (int)blockIdx.x ? v[q] : 0u;
    }
    uint32_t pre;
    block_exclusive_scan(before, lds, pre);
    block_exclusive_scan(every, lds, all);
    return pre;
}

__global__ void __launch_bounds__(kScanBlock)
k_scan_apply(const uint32_t *__restrict__ counts, const uint32_t *__restrict__ idx, const uint32_t *__restrict__ n_dev,
             int64_t n_max, int flag, const uint32_t *__restrict__ part, uint32_t *__restrict__ out,
             uint32_t *__restrict__ total, uint32_t *__restrict__ clear) {
    __shared__ uint32_t lds[kScanBlock / kWave];
    const int64_t n = scan_n(n_dev, n_max);
    const int64_t chunk = scan_chunk(n);
    const int64_t b0 = (int64_t)blockIdx.x * chunk < n ? (int64_t)blockIdx.x * chunk : n;
    const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
    uint32_t all;
    uint32_t running = partial_prefix(part, lds, all);
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *total = all;
        if (clear) *clear = 0u;  // a counter of the next kernel, cleared here to save a launch
    }
    for (int64_t base = b0; base < b1; base += kScanTile) {
        uint32_t v[kScanItems];
        uint32_t sum = 0;
        const int64_t p0 = base + (int64_t)threadIdx.x * kScanItems;
        const bool whole = p0 + kScanItems <= b1;
        if (whole && !idx && flag == 0) {  // two 16-byte loads
            const uint4 a = *reinterpret_cast<const uint4 *>(counts + p0);
            const uint4 b = *reinterpret_cast<const uint4 *>(counts + p0 + 4);
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        } else {
#pragma unroll
            for (int k = 0; k < kScanItems; ++k) {
                const int64_t p = p0 + k;
                v[k] = p < b1 ? load_count(counts, idx, p, flag) : 0u;
            }
        }
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) sum += v[k];
        uint32_t tot;
        uint32_t pre = running + block_exclusive_scan(sum, lds, tot);
        uint32_t o[kScanItems];
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            o[k] = pre;
            pre += v[k];
        }
        if (whole) {
            *reinterpret_cast<uint4 *>(out + p0) = make_uint4(o[0], o[1], o[2], o[3]);
            *reinterpret_cast<uint4 *>(out + p0 + 4) = make_uint4(o[4], o[5], o[6], o[7]);
        } else {
#pragma unroll
            for (int k = 0; k < kScanItems; ++k)
                if (p0 + k < b1) out[p0 + k] = o[k];
        }
        running += tot;
    }
}

// The flag scan's second half fused with the compaction: the records with counts[r] != 0
// go to consecutive positions in record order, with the depth key in ckey and the record
// index (with pack, also its pair count) in cval.  Same chunking as k_scan_reduce; part
// holds each block's count of live records (k_scan_reduce's), and *n_live gets their sum.  Element base + 256 k + t of a
// tile is thread t's k-th: every load and store instruction covers consecutive words, and
// a live record's position is the live count of earlier (row, wave) groups plus its rank
// among its wave's live lanes (a ballot).
__global__ void __launch_bounds__(kScanBlock)
k_scan_compact(const uint32_t *__restrict__ counts, const uint32_t *__restrict__ dkey, int64_t n,
               const uint32_t *__restrict__ part, uint32_t *__restrict__ ckey, uint32_t *__restrict__ cval,
               int pack, uint32_t *__restrict__ n_live) {
    constexpr int NW = kScanBlock / kWave;
    __shared__ uint32_t gcnt[kScanItems][NW];  // live records per (row, wave)
    __shared__ uint32_t lds[kScanBlock / kWave];
    const int64_t chunk = scan_chunk(n);
    const int64_t b0 = (int64_t)blockIdx.x * chunk < n ? (int64_t)blockIdx.x * chunk : n;
    const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
    const int wid = threadIdx.x / kWave, lane = lane_id();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t all;
    uint32_t running = partial_prefix(part, lds, all);
    if (threadIdx.x == 0 && blockIdx.x == 0) *n_live = all;
    for (int64_t base = b0; base < b1; base += kScanTile) {
        uint32_t c[kScanItems], dk[kScanItems];
        uint64_t m[kScanItems];
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int64_t p = base + k * kScanBlock + threadIdx.x;
            c[k] = p < b1 ? counts[p] : 0u;
            dk[k] = p < b1 ? dkey[p] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            m[k] = ballot(c[k] != 0u);
            if (lane == 0) gcnt[k][wid] = (uint32_t)__popcll(m[k]);
        }
        __syncthreads();
        uint32_t pre[kScanItems], acc = 0u;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            for (int w = 0; w < NW; ++w) {
                if (w == wid) pre[k] = acc;
                acc += gcnt[k][w];
            }
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (c[k] == 0u) continue;
            const int64_t p = base + k * kScanBlock + threadIdx.x;
            const uint32_t pos = running + pre[k] + (uint32_t)__popcll(m[k] & lt);
            ckey[pos] = dk[k];
            cval[pos] = pack ? (uint32_t)p | (min(c[k], kPackCountMax) << kPackShift) : (uint32_t)p;
        }
        running += acc;
        __syncthreads();  // the counts are read before the next tile writes them
    }
}

// ------------------------------- radix sort -------------------------------------------
//
// LSD radix sort with one histogram pass for every digit and one kernel per digit pass
// (the single-sweep scheme with decoupled look-back of Merrill and Garland's scan and
// Adinets and Merrill's Onesweep sort).  Keys are cut into tiles of 8192 (8 waves x 16
// steps of 64).  Block b of a pass kernel ranks tile b's keys stably (wave-level match of
// equal digits by ballots, then per-digit offsets across the eight waves).  In the first
// pass the count of each digit in all earlier tiles comes from the histogram kernel,
// which counts the first digit per tile, and a scan of those counts.  Later passes see
// the tiles in an order only the previous pass knows: block b publishes its per-digit
// counts and finds the earlier tiles' counts by walking back over their published words
// until one carries an inclusive prefix; it then publishes its own inclusive prefix.  Workgroups are dispatched in index order, so a
// block only waits for blocks that are already running, which never wait for later ones:
// the walk ends.  (Taking tile numbers from a global counter instead would serialise the
// blocks on one atomic address, tens of nanoseconds each.)  A wait is still bounded (then
// the sort is abandoned and the stall flag set) so that a broken ordering assumption or
// a fault elsewhere cannot leave the kernel spinning.  The tile is staged in LDS in sorted order and
// written so that consecutive lanes write consecutive addresses within each digit's run;
// its keys and then its values pass through one array, so that a block needs about 40 KB
// of LDS and, at 80 VGPRs, three blocks share a CU (two when both were staged at once:
// the last of the tiles then ran as a second, mostly empty round of blocks).
// The key count may be read from device memory; only its ceil(n / 8192) tiles are used.

constexpr int kSortBlock = 512;
constexpr int kSortWaves = kSortBlock / kWave;
constexpr int kSortSteps = 16;
constexpr int kSortTile = kSortBlock * kSortSteps;  // 8192 keys (fewer tiles to look back over)
constexpr int kSortMaxPasses = 8;
// Published word per (tile, digit): flag in bits 31:30, count in bits 29:0.
constexpr uint32_t kStatAgg = 1u << 30;  // the tile's own count
constexpr uint32_t kStatInc = 2u << 30;  // count over this and every earlier tile
constexpr uint32_t kStatCount = (1u << 30) - 1u;
constexpr uint32_t kSortSpinLimit = 1u << 20;
constexpr int kLookback = 8;  // earlier tiles read per look-back step (16 and 32 measured slower)
constexpr int kHistBlocks = 1024;

__device__ inline int64_t sort_count(const uint32_t *n_dev, int64_t n_max) {
    if (!n_dev) return n_max;
    const int64_t n = (int64_t)*n_dev;
    return n < n_max ? n : n_max;
}

// Tiles holding the n live keys.
__device__ inline int64_t sort_active_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

// Per-block digit counts of the later passes (bhist) and the first pass's per-tile digit
// counts (tcount[d * tstride + tile]): a block takes whole tiles, so the first pass finds
// each tile's offsets by a scan of these counts (k_radix_tile_prefix) instead of by
// look-back.  Later passes read tiles in an order that only the pass before them knows,
// so they keep the look-back.
template <int DB>
__global__ void __launch_bounds__(kSortBlock)
k_radix_hist(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ n_dev, int64_t n_max, int passes,
             uint32_t *__restrict__ bhist, uint32_t *__restrict__ tcount, int64_t tstride) {
    constexpr int R = 1 << DB;
    constexpr int kCopies = 4;
    __shared__ uint32_t h[kSortMaxPasses * R * kCopies];
    __shared__ uint32_t tc[kSortWaves][R];  // this tile's first-pass digits, one row per wave
    const int wid = threadIdx.x / kWave, lane = lane_id();
    // The later passes' counters, kCopies interleaved copies of each, lane l adding to copy
    // l % kCopies. High digits take few values within a wave (the exponent and top mantissa
    // bits of depths; the tile row of one Gaussian's tiles), so most lanes would add to one
    // counter and the LDS atomics would serialise.
    for (int i = threadIdx.x; i < passes * R * kCopies; i += kSortBlock) h[i] = 0u;
    const int64_t n = sort_count(n_dev, n_max);
    const int64_t tiles = sort_active_tiles(n);
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        for (int d = lane; d < R; d += kWave) tc[wid][d] = 0u;
        __syncthreads();
        const int64_t b = tile * kSortTile + threadIdx.x;
        uint32_t k[kSortSteps];
#pragma unroll
        for (int st = 0; st < kSortSteps; ++st) k[st] = b + st * kSortBlock < n ? keys[b + st * kSortBlock] : 0u;
#pragma unroll
        for (int st = 0; st < kSortSteps; ++st) {
            if (b + st * kSortBlock >= n) continue;
            atomicAdd(&tc[wid][k[st] & (R - 1)], 1u);
            for (int p = 1; p < passes; ++p)
                atomicAdd(&h[(p * R + ((k[st] >> (p * DB)) & (R - 1))) * kCopies + (lane & (kCopies - 1))], 1u);
        }
        __syncthreads();
        for (int d = threadIdx.x; d < R; d += kSortBlock) {
            uint32_t c = 0u;
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) c += tc[w][d];
            tcount[d * tstride + tile] = c;
        }
        __syncthreads();  // the rows are read before the next tile clears them
    }
    __syncthreads();
    // This block's counts of the later passes' digits (summed over the blocks by
    // k_radix_tile_prefix: plain stores, where atomics from every block on the same few
    // hundred words would queue behind each other).
    for (int i = R + threadIdx.x; i < passes * R; i += kSortBlock) {
        uint32_t t = 0u;
#pragma unroll
        for (int c = 0; c < kCopies; ++c) t += h[i * kCopies + c];
        bhist[(int64_t)blockIdx.x * passes * R + i] = t;
    }
}

// Exclusive prefix over the tiles of each first-pass digit's per-tile counts, in place:
// block d scans row d and writes the digit's total to ghist[d]; it also sums digit d of
// every later pass over the histogram blocks' partial counts into ghist[p R + d].
template <int DB>
__global__ void __launch_bounds__(kScanBlock)
k_radix_tile_prefix(uint32_t *__restrict__ tcount, int64_t tstride, const uint32_t *__restrict__ n_dev,
                    int64_t n_max, int passes, const uint32_t *__restrict__ bhist, int hist_blocks,
                    uint32_t *__restrict__ ghist) {
    constexpr int R = 1 << DB;
    __shared__ uint32_t lds[kScanBlock / kWave];
    const int d = blockIdx.x;
    // Every partial is loaded before any is added (one memory latency, not one per block).
    uint32_t c[kSortMaxPasses] = {};
#pragma unroll
    for (int j = 0; j < kHistBlocks / kScanBlock; ++j) {
        const int b = threadIdx.x + j * kScanBlock;
#pragma unroll
        for (int p = 1; p < kSortMaxPasses; ++p)
            if (p < passes && b < hist_blocks) c[p] += bhist[((int64_t)b * passes + p) * R + d];
    }
#pragma unroll
    for (int p = 1; p < kSortMaxPasses; ++p) {
        if (p >= passes) break;
        uint32_t tot;
        block_exclusive_scan(c[p], lds, tot);
        if (threadIdx.x == 0) ghist[p * R + d] = tot;
    }
    const int64_t tiles = sort_active_tiles(sort_count(n_dev, n_max));
    uint32_t *row = tcount + blockIdx.x * tstride;
    uint32_t running = 0u;
    for (int64_t base = 0; base < tiles; base += kScanTile) {
        uint32_t v[kScanItems];
        uint32_t sum = 0u;
        const int64_t t0 = base + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
        for (int q = 0; q < kScanItems; ++q) {
            v[q] = t0 + q < tiles ? row[t0 + q] : 0u;
            sum += v[q];
        }
        uint32_t tot;
        uint32_t pre = running + block_exclusive_scan(sum, lds, tot);
#pragma unroll
        for (int q = 0; q < kScanItems; ++q) {
            if (t0 + q < tiles) row[t0 + q] = pre;
            pre += v[q];
        }
        running += tot;
    }
    if (threadIdx.x == 0) ghist[d] = running;
}

__device__ inline uint32_t load_status(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_status(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int DB>
__global__ void __launch_bounds__(kSortBlock) __attribute__((amdgpu_waves_per_eu(6)))  // 3 blocks per CU
k_radix_pass(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
             uint32_t *__restrict__ vout, const uint32_t *__restrict__ n_dev, int64_t n_max, int shift,
             const uint32_t *__restrict__ ghist, uint32_t *__restrict__ status,
             uint32_t *__restrict__ status_next, uint32_t *__restrict__ stall, uint2 *__restrict__ ranges,
             const uint32_t *__restrict__ tprefix, int64_t tstride) {
    constexpr int R = 1 << DB;
    __shared__ uint32_t wcnt[kSortWaves][R];
    __shared__ uint32_t dstart[R];
    __shared__ uint32_t dcount[R];
    __shared__ uint32_t gbase[R];
    __shared__ uint32_t scan_lds[kSortWaves];
    __shared__ uint32_t lk[kSortTile];  // the tile in sorted order: keys, then values
    const int wid = threadIdx.x / kWave, lane = lane_id();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t n = sort_count(n_dev, n_max);
    const int64_t tile = blockIdx.x;
    if (tile >= sort_active_tiles(n)) return;  // block-uniform
    const uint32_t gcount = threadIdx.x < R ? ghist[threadIdx.x] : 0u;
    // With tprefix: the digit's count in all earlier tiles, loaded now so that its latency
    // passes while the tile is ranked.
    const uint32_t tpre = tprefix && threadIdx.x < R ? tprefix[threadIdx.x * tstride + tile] : 0u;
    for (int d = lane; d < R; d += kWave) wcnt[wid][d] = 0u;
    __builtin_amdgcn_wave_barrier();
    const int64_t tile_begin = tile * kSortTile;
    const int64_t b = tile_begin + (int64_t)wid * (kSortTile / kSortWaves);
    uint32_t key[kSortSteps], val[kSortSteps], rank[kSortSteps];
    // All key loads first, so that the tile is in flight at once rather than one step at a time.
#pragma unroll
    for (int st = 0; st < kSortSteps; ++st) {
        const int64_t i = b + st * kWave + lane;
        key[st] = i < n ? kin[i] : 0u;
    }
#pragma unroll
    for (int st = 0; st < kSortSteps; ++st) {
        const bool act = b + st * kWave + lane < n;
        const uint32_t d = (key[st] >> shift) & (R - 1);
        const uint64_t a = ballot(act);
        uint32_t mlo = (uint32_t)a, mhi = (uint32_t)(a >> 32);
#pragma unroll
        for (int bit = 0; bit < DB; ++bit) {
            // t is all ones where the bit is set: the lanes agreeing with this one are
            // ballot ^ ~t.
            const uint32_t t = (uint32_t)(((int32_t)(d << (31 - bit))) >> 31);
            const uint64_t bb = ballot(t != 0u);
            mlo &= ~((uint32_t)bb ^ t);
            mhi &= ~((uint32_t)(bb >> 32) ^ t);
        }
        const uint64_t m = ((uint64_t)mhi << 32) | mlo;
        rank[st] = 0xffffffffu;
        if (act) {
            const uint32_t r = (uint32_t)__popcll(m & lt);
            const uint32_t base_d = wcnt[wid][d];
            rank[st] = base_d + r;
            if (r == 0) wcnt[wid][d] = base_d + (uint32_t)__popcll(m);
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // Per digit: offsets of the four waves and the tile's count, published at once.
    uint32_t tot = 0;
    if (threadIdx.x < R) {
        const int d = threadIdx.x;
        uint32_t acc = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            const uint32_t c = wcnt[w][d];
            wcnt[w][d] = acc;
            acc += c;
        }
        tot = acc;
        if (!tprefix) store_status(status + tile * R + d, (tile == 0 ? kStatInc : kStatAgg) | tot);
        status_next[tile * R + d] = 0u;  // the next pass's word for this tile
    }
    uint32_t all;
    const uint32_t gpre = block_exclusive_scan<kSortWaves>(gcount, scan_lds, all);
    const uint32_t pre = block_exclusive_scan<kSortWaves>(tot, scan_lds, all);
    if (threadIdx.x < R) {
        dstart[threadIdx.x] = pre;
        dcount[threadIdx.x] = tot;
    }
    __syncthreads();
    // The keys go to their place in the sorted tile now (it depends on this tile alone), and
    // the values are loaded: fewer registers are live through the look-back, and the loads'
    // latency passes during it. rank[] becomes the position in the sorted tile.
#pragma unroll
    for (int st = 0; st < kSortSteps; ++st) {
        if (rank[st] == 0xffffffffu) continue;
        const uint32_t d = (key[st] >> shift) & (R - 1);
        rank[st] += dstart[d] + wcnt[wid][d];
        lk[rank[st]] = key[st];
    }
#pragma unroll
    for (int st = 0; st < kSortSteps; ++st) {
        const int64_t i = b + st * kWave + lane;
        val[st] = i < n ? vin[i] : 0u;
    }
    if (threadIdx.x < R) {
        const int d = threadIdx.x;
        uint32_t prefix = 0;
        if (tprefix) {
            prefix = tpre;
        } else if (tile > 0) {
            // Words of kLookback earlier tiles are read at once (one memory latency per
            // window instead of per tile), then taken nearest first.
            int64_t j = tile - 1;
            uint32_t spins = 0;
            for (;;) {
                uint32_t w[kLookback];
#pragma unroll
                for (int q = 0; q < kLookback; ++q)
                    w[q] = j - q >= 0 ? load_status(status + (j - q) * R + d) : kStatInc;
                int used = kLookback;
                bool done = false;
#pragma unroll
                for (int q = 0; q < kLookback; ++q) {
                    if (q < used && !done) {
                        if ((w[q] & ~kStatCount) == 0u) {
                            used = q;  // not yet published: read again from this tile
                        } else {
                            prefix += w[q] & kStatCount;
                            done = (w[q] & kStatInc) != 0u;  // tile 0's word is inclusive
                        }
                    }
                }
                if (done) break;
                j -= used;
                if (used < kLookback) {
                    if (++spins > kSortSpinLimit || load_status(stall) != 0u) {
                        store_status(stall, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            store_status(status + tile * R + d, kStatInc | (prefix + tot));
        }
        gbase[d] = gpre + prefix;
    }
    __syncthreads();
    // The sorted keys are read back (key[] now holds them in the tile's sorted order) before
    // the values take their place in the same array: half the LDS of staging both at once,
    // so that three blocks fit on a CU.
    const int cnt = (int)(n - tile_begin < kSortTile ? n - tile_begin : kSortTile);
#pragma unroll
    for (int st = 0; st < kSortSteps; ++st) {
        const int j = threadIdx.x + st * kSortBlock;
        if (j >= cnt) continue;
        const uint32_t k = lk[j];
        key[st] = k;
        if (ranges) {
            // Final pass over tile ids: the tile is sorted in LDS, so the output neighbours of
            // an element inside its digit's run are its LDS neighbours.  At the ends of the
            // run they belong to other blocks: the first and last element then take the
            // extreme position by atomics (the true start or end, wherever it lies, wins).
            const uint32_t d = (k >> shift) & (R - 1);
            const uint32_t pos = gbase[d] + ((uint32_t)j - dstart[d]);
            const uint32_t first = dstart[d], last = dstart[d] + dcount[d] - 1u;
            if ((uint32_t)j == first) atomicMin(&ranges[k].x, pos);
            else if (lk[j - 1] != k) ranges[k].x = pos;
            if ((uint32_t)j == last) atomicMax(&ranges[k].y, pos + 1u);
            else if (lk[j + 1] != k) ranges[k].y = pos + 1u;
        }
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < kSortSteps; ++st)
        if (rank[st] != 0xffffffffu) lk[rank[st]] = val[st];
    __syncthreads();
#pragma unroll
    for (int st = 0; st < kSortSteps; ++st) {
        const int j = threadIdx.x + st * kSortBlock;
        if (j >= cnt) continue;
        const uint32_t k = key[st];
        const uint32_t d = (k >> shift) & (R - 1);
        const uint32_t pos = gbase[d] + ((uint32_t)j - dstart[d]);
        if (kout) kout[pos] = k;  // the last pass may drop the keys: only the values are used
        vout[pos] = lk[j];
    }
}

// ------------------------------- pairs and ranges -------------------------------------

__device__ inline void emit_row(uint32_t *__restrict__ pkey, uint32_t *__restrict__ pval, uint32_t cap, uint32_t &k,
                                uint32_t base, uint32_t tiles_x, int ty, int ta, int tb, uint32_t r) {
    for (int tx = ta; tx <= tb; ++tx, ++k) {
        if (k >= cap) return;
        pkey[k] = base + (uint32_t)ty * tiles_x + (uint32_t)tx;
        pval[k] = r;
    }
}

// One lane per record (in depth order; sorted_counts[p] is the pair count of sorted_rec[p]).
// Records with many pairs are queued for k_keygen_big.
//
// A wave's records are consecutive in depth order, so their pairs form one contiguous run
// of the output.  The wave lists the tile rows of its records in LDS (output position,
// first global tile, length, record; in output order) and then fills its run 64
// positions at a time, one position per lane: the row that a position falls in is the
// last row starting at or before it, found from the rows starting inside the 64-position
// window (a ballot and a prefix count), so every lane emits one pair per step whatever
// the records' sizes and the stores are consecutive.  Records whose rows the counting pass
// did not cache (more than kSpanRowsMax rows) are emitted by their own lane, row by row;
// positions of queued large records are left to k_keygen_big.
constexpr int kKeygenBlock = 256;
constexpr int kKeygenWaves = kKeygenBlock / kWave;
constexpr int kKeygenRows = kWave * (int)kSpanRowsMax;  // rows of one wave's records, at most

__global__ void __launch_bounds__(kKeygenBlock)
k_keygen(const uint32_t *__restrict__ sorted_rec, uint32_t rec_mask, const uint32_t *__restrict__ sorted_counts,
         const uint32_t *__restrict__ offsets, const float4 *__restrict__ rec, const uint4 *__restrict__ spans,
         RasterSettings rs, int64_t n_records, int64_t n_per_view, ViewTable vt, uint32_t *__restrict__ pkey,
         uint32_t *__restrict__ pval, FrameHeader *__restrict__ hdr, uint32_t cap,
         const uint32_t *__restrict__ total, uint32_t *__restrict__ big_list, uint32_t *__restrict__ big_count,
         const uint32_t *__restrict__ n_dev, uint2 *__restrict__ ranges, int64_t n_tiles) {
    __shared__ uint32_t row_pos[kKeygenWaves][kKeygenRows];   // first output position
    __shared__ uint32_t row_tile[kKeygenWaves][kKeygenRows];  // global tile id of the first tile
    __shared__ uint32_t row_rec[kKeygenWaves][kKeygenRows];   // record index
    __shared__ uint8_t row_len[kKeygenWaves][kKeygenRows];    // tiles (at most kBigRecord)
    __shared__ uint8_t starts[kKeygenWaves][kWave];          // rows starting at window position
    const int wid = threadIdx.x / kWave, lane = lane_id();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // Empty tile ranges, for the tile sort's last pass to narrow (here to save a launch).
    for (int64_t t = p; t < n_tiles; t += (int64_t)gridDim.x * blockDim.x) ranges[t] = make_uint2(0xffffffffu, 0u);
    if (p == 0) {
        // Everything a backward checks before it reads the frame state.
        const uint32_t t = *total;
        hdr->pairs = t;
        hdr->overflow = t > cap ? 1u : 0u;
        hdr->capacity = cap;
        hdr->tile = (uint32_t)vt.tile;
        hdr->n_views = (uint32_t)vt.n_views;
        hdr->n_tiles = (uint32_t)vt.tile_off[vt.n_views];
        hdr->n_pixels = (uint64_t)vt.pix_off[vt.n_views];
        hdr->n_records = (uint64_t)n_records;
        hdr->magic = kFrameMagic;
        hdr->visible = (uint32_t)rs.mark_visible;
        hdr->counted = (uint32_t)rs.count_work;
        hdr->ppt = (uint32_t)vt.ppt;
        hdr->frame = (uint32_t)rs.frame;
        hdr->bwd_error = 0u;
        hdr->walked = hdr->accepted = 0u;
    }
    n_records = scan_n(n_dev, n_records);
    const bool act = p < n_records;
    uint32_t r = 0, c = 0, k = 0;
    if (act) {
        r = sorted_rec[p] & rec_mask;
        c = sorted_counts[p];
        k = offsets[p];
    }
    const bool big = c > kBigRecord;
    const uint32_t slot = wave_append(big_count, big);
    if (big) big_list[slot] = (uint32_t)p;
    const bool own = act && c != 0u && !big;
    int v = 0, ty0 = 0, nr = 0;
    uint32_t base = 0, tiles_x = 0;
    uint4 sp = make_uint4(0u, 0u, 0u, 0u);
    if (own) {
        v = (int)(r / (uint32_t)n_per_view);  // 32-bit: record indices fit
        base = (uint32_t)vt.tile_off[v];
        tiles_x = (uint32_t)vt.tiles_x[v];
        sp = spans[r];
        nr = (int)(sp.x >> 16);
        ty0 = (int)(sp.x & 0xffffu);
    }
    const bool cached = own && nr <= (int)kSpanRowsMax;
    // This lane's non-empty rows, their place in the wave's row list, then the list.
    uint32_t n_rows = 0;
    if (cached) {
        for (int i = 0; i < nr; ++i) {
            int ta, tb;
            span_row(sp, nr, i, ta, tb);
            n_rows += ta <= tb ? 1u : 0u;
        }
    }
    const uint32_t inc = wave_inclusive_scan(n_rows);
    const uint32_t rows_wave = (uint32_t)__shfl((int)inc, kWave - 1, kWave);
    if (cached) {
        uint32_t t = inc - n_rows, pos = k;
        for (int i = 0; i < nr; ++i) {
            int ta, tb;
            span_row(sp, nr, i, ta, tb);
            if (ta > tb) continue;
            row_pos[wid][t] = pos;
            row_tile[wid][t] = base + (uint32_t)(ty0 + i) * tiles_x + (uint32_t)ta;
            row_rec[wid][t] = r;
            row_len[wid][t] = (uint8_t)(tb - ta + 1);
            pos += (uint32_t)(tb - ta + 1);
            ++t;
        }
    } else if (own) {
        // Not cached: this lane evaluates its rows and stores its pairs itself.
        Footprint f;
        if (record_footprint(rec[4 * (int64_t)r], rec[4 * (int64_t)r + 1], rs.alpha_min, vt.width[v], vt.height[v],
                             f)) {
            const int T = vt.tile, sh = __builtin_ctz((unsigned)vt.tile);
            uint32_t kk = k;
            for (int ty = f.j0 >> sh; ty <= f.j1 >> sh; ++ty) {
                int ta, tb;
                if (row_span(f, T, ty, ta, tb)) emit_row(pkey, pval, cap, kk, base, tiles_x, ty, ta, tb, r);
            }
        }
    }
    // The run ends at the largest end of the wave's records (queued ones included); lane 0
    // holds the wave's first record (if it has none, neither has any other lane).
    const uint32_t run0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)k);
    uint32_t end = act ? k + c : run0;
    for (int off = 32; off > 0; off >>= 1) end = max(end, (uint32_t)__shfl_xor((int)end, off, 64));
    if (end > cap) end = cap;
    const uint64_t le = (lane == kWave - 1) ? ~0ull : ((2ull << lane) - 1ull);  // lanes <= this one
    uint32_t before = 0;  // rows starting before the window
    __builtin_amdgcn_wave_barrier();  // the row list is written (one wave's LDS accesses stay in order)
    for (uint32_t j0 = run0; j0 < end; j0 += kWave) {
        starts[wid][lane] = 0;
        __builtin_amdgcn_wave_barrier();
        // Rows are in output order: those starting in this window follow the earlier ones.
        const uint32_t t = before + (uint32_t)lane;
        if (t < rows_wave) {
            const uint32_t s0 = row_pos[wid][t];
            if (s0 < j0 + kWave) starts[wid][s0 - j0] = 1;
        }
        __builtin_amdgcn_wave_barrier();
        const uint64_t m = ballot(starts[wid][lane] != 0);
        const uint32_t j = j0 + (uint32_t)lane;
        const int owner = (int)(before + (uint32_t)__popcll(m & le)) - 1;
        if (owner >= 0 && j < end) {
            const uint32_t d = j - row_pos[wid][owner];
            if (d < (uint32_t)row_len[wid][owner]) {  // else a position of an uncached or queued record
                pkey[j] = row_tile[wid][owner] + d;
                pval[j] = row_rec[wid][owner];
            }
        }
        before += (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();  // the marks are read before the next window clears them
    }
}

__global__ void __launch_bounds__(256)
k_keygen_big(const uint32_t *__restrict__ sorted_rec, uint32_t rec_mask, const uint32_t *__restrict__ offsets,
             const float4 *__restrict__ rec, RasterSettings rs, int64_t n_per_view, ViewTable vt,
             uint32_t *__restrict__ pkey, uint32_t *__restrict__ pval, uint32_t cap,
             const uint32_t *__restrict__ big_list, const uint32_t *__restrict__ big_count) {
    const int lane = lane_id();
    const uint32_t n_big = *big_count;
    const uint32_t n_waves = gridDim.x * (blockDim.x / kWave);
    for (uint32_t w = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; w < n_big; w += n_waves) {
        const uint32_t p = big_list[w];
        const uint32_t r = sorted_rec[p] & rec_mask;
        const int v = (int)(r / (uint32_t)n_per_view);
        Footprint f;
        if (!record_footprint(rec[4 * (int64_t)r], rec[4 * (int64_t)r + 1], rs.alpha_min, vt.width[v],
                              vt.height[v], f))
            continue;  // wave-uniform
        const int T = vt.tile, sh = __builtin_ctz((unsigned)vt.tile);
        const uint32_t base = (uint32_t)vt.tile_off[v], tiles_x = (uint32_t)vt.tiles_x[v];
        uint32_t k0 = offsets[p];
        for (int ty0 = f.j0 >> sh; ty0 <= f.j1 >> sh; ty0 += kWave) {
            const int ty = ty0 + lane;
            int ta = 0, tb = -1;
            if (ty <= f.j1 >> sh && !row_span(f, T, ty, ta, tb)) tb = ta - 1;
            if (ty > f.j1 >> sh) tb = ta - 1;
            const uint32_t len = (uint32_t)(tb - ta + 1);
            const uint32_t inc = wave_inclusive_scan(len);
            uint32_t k = k0 + inc - len;
            if (len) emit_row(pkey, pval, cap, k, base, tiles_x, ty, ta, tb, r);
            k0 += __shfl(inc, kWave - 1, kWave);
        }
    }
}

__global__ void __launch_bounds__(256) k_sum_u64(const uint32_t *__restrict__ x, int64_t n,
                                                unsigned long long *__restrict__ out) {
    unsigned long long acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += x[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane_id() == 0 && acc) atomicAdd(out, acc);
}

}  // namespace

hipError_t launch_sum_u64(const uint32_t *x, int64_t n, unsigned long long *out, hipStream_t s) {
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(out), 0u, 2, s);
    if (e != hipSuccess || n <= 0) return e;
    int64_t nb = (n + 255) / 256;
    if (nb > 1024) nb = 1024;
    hipLaunchKernelGGL(k_sum_u64, dim3((unsigned)nb), dim3(256), 0, s, x, n, out);
    return hipGetLastError();
}

// ------------------------------- host wrappers ----------------------------------------

// One block per tile of kScanTile elements (up to kScanMaxBlocks): every block then does
// one round of loads, scan and stores, where fewer blocks would each wait on several.
static int64_t scan_blocks(int64_t n) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb > kScanMaxBlocks) nb = kScanMaxBlocks;
    return nb < 1 ? 1 : nb;
}

int64_t scan_partials(int64_t n) { return scan_blocks(n); }

hipError_t launch_scan_indirect(const uint32_t *counts, const uint32_t *idx, int64_t n, uint32_t *offsets,
                                uint32_t *total, uint32_t *part, hipStream_t s, const uint32_t *n_dev, int flag,
                                uint32_t *gathered, uint32_t *clear) {
    const int64_t nb = scan_blocks(n);
    // With `gathered`, the reduce pass stores counts[idx[p]] (or its flag) there and the
    // apply pass reads it back contiguously instead of gathering a second time.
    if (!idx) gathered = nullptr;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanBlock), 0, s, counts, idx, n_dev, n, flag, part,
                       gathered);
    if (gathered)
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanBlock), 0, s, gathered, nullptr, n_dev, n, 0,
                           part, offsets, total, clear);
    else
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanBlock), 0, s, counts, idx, n_dev, n, flag,
                           part, offsets, total, clear);
    return hipGetLastError();
}

hipError_t launch_compact(const uint32_t *counts, const uint32_t *dkey, int64_t n, uint32_t *ckey, uint32_t *cval,
                          uint32_t *n_live, uint32_t *part, bool pack, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (pack && n > (int64_t)kPackMask + 1) return hipErrorInvalidValue;
    const int64_t nb = scan_blocks(n);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanBlock), 0, s, counts, nullptr, nullptr, n, 1, part,
                       nullptr);
    hipLaunchKernelGGL(k_scan_compact, dim3((unsigned)nb), dim3(kScanBlock), 0, s, counts, dkey, n, part, ckey, cval,
                       pack ? 1 : 0, n_live);
    return hipGetLastError();
}

static int64_t sort_tiles(int64_t n_max) { return (n_max + kSortTile - 1) / kSortTile; }

// Scratch words: digit histograms [kSortMaxPasses << digit_bits], published words
// [2][tiles << digit_bits] (alternating passes), the first pass's per-tile digit offsets
// [tiles << digit_bits] and the histogram blocks' partial counts.
int64_t radix_hist_words(int64_t n_max, int digit_bits) {
    const int64_t t = sort_tiles(n_max) > 0 ? sort_tiles(n_max) : 1;
    const int64_t hb = t < kHistBlocks ? t : kHistBlocks;
    return ((int64_t)kSortMaxPasses << digit_bits) * (1 + hb) + 3 * (t << digit_bits);
}

template <int DB>
static void sort_passes(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_tmp, uint32_t *vals_tmp,
                        uint32_t *keys_out, uint32_t *vals_out, int64_t n_max, const uint32_t *n_dev, int passes,
                        uint32_t *scratch, uint32_t *stall, uint2 *ranges, bool keep_keys, hipStream_t s) {
    constexpr int R = 1 << DB;
    const int64_t tiles = sort_tiles(n_max);
    uint32_t *ghist = scratch;
    uint32_t *status[2] = {ghist + (int64_t)kSortMaxPasses * R, ghist + (int64_t)kSortMaxPasses * R + tiles * R};
    uint32_t *tprefix = status[1] + tiles * R;  // [R][tiles]: the first pass's per-tile digit offsets
    uint32_t *bhist = tprefix + tiles * R;      // [hist blocks][passes][R]
    int64_t hb = tiles < kHistBlocks ? tiles : kHistBlocks;
    if (hb < 1) hb = 1;
    hipLaunchKernelGGL(k_radix_hist<DB>, dim3((unsigned)hb), dim3(kSortBlock), 0, s, keys_in, n_dev, n_max, passes,
                       bhist, tprefix, tiles);
    hipLaunchKernelGGL(k_radix_tile_prefix<DB>, dim3(R), dim3(kScanBlock), 0, s, tprefix, tiles, n_dev, n_max, passes,
                       bhist, (int)hb, ghist);
    const uint32_t *kin = keys_in, *vin = vals_in;
    for (int p = 0; p < passes; ++p) {
        // The last pass writes to *_out; earlier passes alternate so that this holds.
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        uint32_t *ko = to_out ? keys_out : keys_tmp;
        uint32_t *vo = to_out ? vals_out : vals_tmp;
        hipLaunchKernelGGL(k_radix_pass<DB>, dim3((unsigned)tiles), dim3(kSortBlock), 0, s, kin, vin,
                           p == passes - 1 && !keep_keys ? nullptr : ko, vo, n_dev,
                           n_max, p * DB, ghist + (int64_t)p * R, status[p & 1], status[(p + 1) & 1], stall,
                           p == passes - 1 ? ranges : nullptr, p == 0 ? tprefix : nullptr, tiles);
        kin = ko;
        vin = vo;
    }
}

hipError_t radix_sort(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_tmp, uint32_t *vals_tmp,
                      uint32_t *keys_out, uint32_t *vals_out, int64_t n_max, const uint32_t *n_dev, int bits,
                      int digit_bits, uint32_t *scratch, uint32_t *stall, uint2 *ranges, hipStream_t s,
                      bool keep_keys) {
    if (n_max <= 0) return hipSuccess;
    if (bits < 1) bits = 1;
    if (digit_bits < 4 || digit_bits > 8) return hipErrorInvalidValue;
    // As few passes as digit_bits allows, with the bits spread evenly over them (14 tile-id
    // bits sort as 2 x 7: fewer buckets per pass than 8 + 6).
    const int passes = (bits + digit_bits - 1) / digit_bits;
    if (passes > kSortMaxPasses) return hipErrorInvalidValue;
    int db = (bits + passes - 1) / passes;
    if (db < 4) db = 4;
    switch (db) {
        case 4: sort_passes<4>(keys_in, vals_in, keys_tmp, vals_tmp, keys_out, vals_out, n_max, n_dev, passes, scratch, stall, ranges, keep_keys, s); break;
        case 5: sort_passes<5>(keys_in, vals_in, keys_tmp, vals_tmp, keys_out, vals_out, n_max, n_dev, passes, scratch, stall, ranges, keep_keys, s); break;
        case 6: sort_passes<6>(keys_in, vals_in, keys_tmp, vals_tmp, keys_out, vals_out, n_max, n_dev, passes, scratch, stall, ranges, keep_keys, s); break;
        case 7: sort_passes<7>(keys_in, vals_in, keys_tmp, vals_tmp, keys_out, vals_out, n_max, n_dev, passes, scratch, stall, ranges, keep_keys, s); break;
        default: sort_passes<8>(keys_in, vals_in, keys_tmp, vals_tmp, keys_out, vals_out, n_max, n_dev, passes, scratch, stall, ranges, keep_keys, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_keygen(const uint32_t *sorted_rec, uint32_t rec_mask, const uint32_t *sorted_counts,
                         const uint32_t *offsets, const float *records, const uint4 *spans, const RasterSettings &rs,
                         int64_t n_records, int64_t n_per_view,
                         const ViewTable &vt, uint32_t *pkey, uint32_t *pval, FrameHeader *hdr, uint32_t capacity,
                         const uint32_t *total, uint32_t *big_list, uint32_t *big_count, const uint32_t *n_dev,
                         uint2 *ranges, int64_t n_tiles, hipStream_t s) {
    const float4 *rec = reinterpret_cast<const float4 *>(records);
    const int64_t nb = n_records > 0 ? (n_records + 255) / 256 : 1;
    hipLaunchKernelGGL(k_keygen, dim3((unsigned)nb), dim3(256), 0, s, sorted_rec, rec_mask, sorted_counts, offsets, rec,
                       spans, rs, n_records, n_per_view, vt, pkey, pval, hdr, capacity, total, big_list, big_count,
                       n_dev, ranges, n_tiles);
    if (n_records > 0)
        hipLaunchKernelGGL(k_keygen_big, dim3(1024), dim3(256), 0, s, sorted_rec, rec_mask, offsets, rec, rs,
                           n_per_view, vt, pkey, pval, capacity, big_list, big_count);
    return hipGetLastError();
}

// One workgroup: counting sort of the tiles into 256 work classes (32 list entries each,
// the last one open-ended), heaviest class first.  The order inside a class is that of
// the atomics; any order is a valid launch order.  Each tile is handled by the same
// thread in both loops, so the reset of an empty range is seen by the second.
constexpr int kOrderBlock = 1024;
constexpr int kOrderClasses = 256;
constexpr int kOrderShift = 5;
constexpr int kOrderItems = 8;

__global__ void __launch_bounds__(kOrderBlock)
k_order_tiles(uint2 *__restrict__ ranges, const uint32_t *__restrict__ work, int64_t n,
              uint32_t *__restrict__ order) {
    __shared__ uint32_t cnt[kOrderClasses];
    __shared__ uint32_t scan_lds[kOrderBlock / kWave];
    for (int b = threadIdx.x; b < kOrderClasses; b += kOrderBlock) cnt[b] = 0u;
    __syncthreads();
    auto cls_of = [&](uint32_t w) {
        return (uint32_t)(kOrderClasses - 1) - min((uint32_t)(kOrderClasses - 1), w >> kOrderShift);
    };
    // kOrderItems tiles per thread and step, their reads issued together: one memory latency
    // per step rather than one per tile.
    for (int64_t t0 = threadIdx.x; t0 < n; t0 += (int64_t)kOrderBlock * kOrderItems) {
        uint2 rg[kOrderItems];
        uint32_t wk[kOrderItems];
#pragma unroll
        for (int q = 0; q < kOrderItems; ++q) {
            const int64_t t = t0 + (int64_t)q * kOrderBlock;
            rg[q] = ranges && t < n ? ranges[t] : make_uint2(0u, 0u);
            wk[q] = !ranges && t < n ? work[t] : 0u;
        }
#pragma unroll
        for (int q = 0; q < kOrderItems; ++q) {
            const int64_t t = t0 + (int64_t)q * kOrderBlock;
            if (t >= n) continue;
            if (ranges && rg[q].x > rg[q].y) {
                rg[q] = make_uint2(0u, 0u);
                ranges[t] = rg[q];
            }
            atomicAdd(&cnt[cls_of(ranges ? rg[q].y - rg[q].x : wk[q])], 1u);
        }
    }
    __syncthreads();
    // Class starts: a block-wide scan (one class per thread), not a serial loop of 256
    // dependent LDS round trips.
    uint32_t total;
    const uint32_t c = threadIdx.x < kOrderClasses ? cnt[threadIdx.x] : 0u;
    const uint32_t start = block_exclusive_scan<kOrderBlock / kWave>(c, scan_lds, total);
    if (threadIdx.x < kOrderClasses) cnt[threadIdx.x] = start;
    __syncthreads();
    for (int64_t t0 = threadIdx.x; t0 < n; t0 += (int64_t)kOrderBlock * kOrderItems) {
        uint32_t wk[kOrderItems];
#pragma unroll
        for (int q = 0; q < kOrderItems; ++q) {
            const int64_t t = t0 + (int64_t)q * kOrderBlock;
            if (t < n) {
                const uint2 r = ranges ? ranges[t] : make_uint2(0u, 0u);
                wk[q] = ranges ? r.y - r.x : work[t];
            }
        }
#pragma unroll
        for (int q = 0; q < kOrderItems; ++q) {
            const int64_t t = t0 + (int64_t)q * kOrderBlock;
            if (t < n) order[atomicAdd(&cnt[cls_of(wk[q])], 1u)] = (uint32_t)t;
        }
    }
}

hipError_t launch_order_tiles(uint2 *ranges, const uint32_t *work, int64_t n_tiles, uint32_t *order,
                              hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    if ((ranges == nullptr) == (work == nullptr)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_order_tiles, dim3(1), dim3(kOrderBlock), 0, s, ranges, work, n_tiles, order);
    return hipGetLastError();
}

}  // namespace gspm
