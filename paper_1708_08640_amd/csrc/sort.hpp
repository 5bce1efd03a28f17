// Bind-time primitives of the det-mode build: a stable device-wide LSD radix
// sort of (key, value) pairs, prefix sums, and per-row entry counts.
//
// The sort is what fixes the det order of every sum (the items of a batch in
// item-order position, each row's contributions in position order), so it
// must be stable; each pass is:
//   k_radix_hist     one 256-bin digit histogram per tile of 4,096 items,
//                    stored digit-major ([digit][tile]);
//   scan_i32         exclusive prefix sum of that array: the first output
//                    position of every (digit, tile);
//   k_radix_scatter  the tile again, 256 items per step in input order; a
//                    lane's rank among the equal digits of lower lanes comes
//                    from ballots (one per digit bit), the wavefronts before
//                    it from per-wavefront digit counts in LDS.
// Keys are sorted on bits [0, bits) only, in passes of at most 8 bits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace s3 {

constexpr int kSortThreads = 256;
constexpr int kSortSteps = 16;
constexpr int64_t kSortTile = (int64_t)kSortThreads * kSortSteps;  // items per tile
constexpr int kScanTile = 4096;                                      // values per scan tile

// lanes of this wavefront whose `bits` low bits of d equal this lane's, among
// the lanes with `valid` set (every lane of the wavefront must call it)
__device__ inline uint64_t match_bits(uint32_t d, bool valid, int bits) {
    uint64_t m = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
        const bool on = (d >> b) & 1u;
        const uint64_t v = __ballot(on);
        m &= on ? v : ~v;
    }
    return m;
}

template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K *__restrict__ key, int64_t n, int shift,
                                                           int dbits, int64_t ntiles, int32_t *__restrict__ hist) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t tile = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const uint32_t dmask = (1u << dbits) - 1u;
    for (int i = 0; i < kSortSteps; ++i) {
        const int64_t e = tile * kSortTile + (int64_t)i * kSortThreads + threadIdx.x;
        const bool valid = e < n;
        const uint32_t d = valid ? (uint32_t)(key[e] >> shift) & dmask : 0u;
        const uint64_t m = match_bits(d, valid, dbits);
        if (valid && lane == __ffsll((unsigned long long)m) - 1) atomicAdd(&h[d], __popcll(m));
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + tile] = h[threadIdx.x];
}

template <typename K, typename V>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const K *__restrict__ kin, const V *__restrict__ vin,
                                                              K *__restrict__ kout, V *__restrict__ vout, int64_t n,
                                                              int shift, int dbits, int64_t ntiles,
                                                              const int32_t *__restrict__ first) {
    __shared__ int32_t run[256];      // next output position per digit
    __shared__ int32_t wcnt[4][256];  // this step's digit counts per wavefront
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t tile = blockIdx.x;
    const uint32_t dmask = (1u << dbits) - 1u;
    run[threadIdx.x] = first[(int64_t)threadIdx.x * ntiles + tile];
    for (int i = 0; i < kSortSteps; ++i) {
#pragma unroll
        for (int u = 0; u < 4; ++u) wcnt[u][threadIdx.x] = 0;
        __syncthreads();
        const int64_t e = tile * kSortTile + (int64_t)i * kSortThreads + threadIdx.x;
        const bool valid = e < n;
        K k{};
        V v{};
        if (valid) {
            k = kin[e];
            v = vin[e];
        }
        const uint32_t d = valid ? (uint32_t)(k >> shift) & dmask : 0u;
        const uint64_t m = match_bits(d, valid, dbits);
        const int below = __popcll(m & ((1ull << lane) - 1ull));
        if (valid && below == 0) wcnt[w][d] = __popcll(m);
        __syncthreads();
        if (valid) {
            int64_t pos = run[d] + below;
            for (int u = 0; u < w; ++u) pos += wcnt[u][d];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        run[threadIdx.x] += wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] + wcnt[2][threadIdx.x] + wcnt[3][threadIdx.x];
        __syncthreads();
    }
}

// Prefix sums of int32 values, tile by tile: each tile of kScanTile values is
// scanned in LDS (16 consecutive values per lane, then across lanes); its
// total goes to tile_sum, whose exclusive scan k_scan_add adds back.
__device__ inline int lds_pad(int j) { return j + (j >> 5); }

static __global__ __launch_bounds__(256) void k_scan_tiles(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                                           int64_t n, int exclusive, int32_t *__restrict__ tile_sum) {
    __shared__ int32_t s[kScanTile + kScanTile / 32];
    __shared__ int32_t wsum[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int j = threadIdx.x; j < kScanTile; j += 256) s[lds_pad(j)] = (base + j < n) ? in[base + j] : 0;
    __syncthreads();
    int32_t v[16], acc = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        v[i] = s[lds_pad(threadIdx.x * 16 + i)];
        acc += v[i];
    }
    int32_t inc = acc;  // inclusive scan of lane totals within the wavefront
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int32_t before = inc - acc;
    for (int u = 0; u < w; ++u) before += wsum[u];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int32_t x = v[i];
        s[lds_pad(threadIdx.x * 16 + i)] = exclusive ? before : before + x;
        before += x;
    }
    if (threadIdx.x == 255 && tile_sum) tile_sum[blockIdx.x] = before;
    __syncthreads();
    for (int j = threadIdx.x; j < kScanTile; j += 256)
        if (base + j < n) out[base + j] = s[lds_pad(j)];
}

static __global__ void k_scan_add(int32_t *__restrict__ out, int64_t n, const int32_t *__restrict__ tile_first) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int32_t add = tile_first[blockIdx.x];
    for (int j = threadIdx.x; j < kScanTile; j += blockDim.x)
        if (base + j < n) out[base + j] += add;
}

// Working memory of scan_i32 over n values (the tile sums of every level).
inline size_t scan_temp_elems(int64_t n) {
    size_t total = 0;
    while (n > kScanTile) {
        n = (n + kScanTile - 1) / kScanTile;
        total += (size_t)n;
    }
    return total;
}

// out = inclusive (or exclusive) prefix sum of in (may alias); temp holds
// scan_temp_elems(n) values.
inline hipError_t scan_i32(const int32_t *in, int32_t *out, int64_t n, bool exclusive, int32_t *temp,
                           hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 1) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(256), 0, st, in, out, n, exclusive ? 1 : 0,
                           (int32_t *)nullptr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(256), 0, st, in, out, n, exclusive ? 1 : 0, temp);
    hipError_t e = scan_i32(temp, temp, tiles, true, temp + tiles, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(256), 0, st, out, n, (const int32_t *)temp);
    return hipGetLastError();
}

// Working memory of radix_sort_pairs over n items, in bytes.
inline size_t sort_temp_bytes(int64_t n) {
    const int64_t tiles = (n + kSortTile - 1) / kSortTile;
    return sizeof(int32_t) * ((size_t)256 * tiles + scan_temp_elems(256 * tiles));
}

// Stable sort of (kin, vin) by bits [0, bits) of the keys into (kout, vout).
// kin and vin are overwritten (they serve as the second buffer); n < 2^31.
template <typename K, typename V>
hipError_t radix_sort_pairs(K *kin, V *vin, K *kout, V *vout, int64_t n, int bits, void *temp, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (n + kSortTile - 1) / kSortTile;
    int32_t *hist = (int32_t *)temp;
    int32_t *stemp = hist + 256 * tiles;
    const int passes = bits <= 0 ? 1 : (bits + 7) / 8;
    K *ks = kin, *kd = kout;
    V *vs = vin, *vd = vout;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * 8;
        const int dbits = bits <= 0 ? 1 : ((bits - shift) < 8 ? (bits - shift) : 8);
        hipLaunchKernelGGL((k_radix_hist<K>), dim3((unsigned)tiles), dim3(kSortThreads), 0, st, (const K *)ks, n,
                           shift, dbits, tiles, hist);
        hipError_t e = scan_i32(hist, hist, 256 * tiles, true, stemp, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_radix_scatter<K, V>), dim3((unsigned)tiles), dim3(kSortThreads), 0, st, (const K *)ks,
                           (const V *)vs, kd, vd, n, shift, dbits, tiles, (const int32_t *)hist);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        K *tk = ks; ks = kd; kd = tk;
        V *tv = vs; vs = vd; vd = tv;
    }
    if (ks != kout) {  // an even number of passes ends in the input buffers
        hipError_t e = hipMemcpyAsync(kout, ks, sizeof(K) * n, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(vout, vs, sizeof(V) * n, hipMemcpyDeviceToDevice, st);
        return e;
    }
    return hipSuccess;
}

// Bits needed for values in [0, limit).
inline int bits_for(uint64_t limit) {
    int b = 0;
    while (b < 64 && (limit - 1) >> b) ++b;
    return b;
}

// Row counts.  Power-law indices make plain per-entry atomics serialise on
// the head rows, so the lanes of a wavefront holding the same index (matched
// by ballots over its `bits` low bits) add their count once.
static __global__ __launch_bounds__(256) void k_hist(const int32_t *__restrict__ idx, int64_t n, int bits,
                                                     int32_t *__restrict__ cnt) {
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // every lane of a wavefront runs the same number of iterations
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    for (int64_t b0 = first; b0 < n; b0 += stride) {
        const int64_t e = b0 + lane;
        const bool valid = e < n;
        const uint32_t v = valid ? (uint32_t)idx[e] : 0u;
        const uint64_t m = match_bits(v, valid, bits);
        if (valid && lane == __ffsll((unsigned long long)m) - 1) atomicAdd(&cnt[v], __popcll(m));
    }
}

// The same for modes of at most kHistLdsRows rows: counts gather in an LDS
// histogram per workgroup first, then one global add per row and workgroup.
constexpr int kHistLdsRows = 8192;

static __global__ __launch_bounds__(256) void k_hist_lds(const int32_t *__restrict__ idx, int64_t n, int rows,
                                                         int bits, int32_t *__restrict__ cnt) {
    __shared__ int32_t h[kHistLdsRows];
    for (int r = threadIdx.x; r < rows; r += blockDim.x) h[r] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    for (int64_t b0 = first; b0 < n; b0 += stride) {
        const int64_t e = b0 + lane;
        const bool valid = e < n;
        const uint32_t v = valid ? (uint32_t)idx[e] : 0u;
        const uint64_t m = match_bits(v, valid, bits);
        if (valid && lane == __ffsll((unsigned long long)m) - 1) atomicAdd(&h[v], __popcll(m));
    }
    __syncthreads();
    for (int r = threadIdx.x; r < rows; r += blockDim.x)
        if (h[r]) atomicAdd(&cnt[r], h[r]);
}

// cnt[r] += number of entries of idx equal to r, for r in [0, rows)
inline void row_counts(const int32_t *idx, int64_t n, int64_t rows, int32_t *cnt, hipStream_t st) {
    if (n <= 0) return;
    const int bits = bits_for((uint64_t)rows);
    int64_t g = (n + 255) / 256;
    if (rows <= kHistLdsRows) {
        if (g > 1024) g = 1024;
        hipLaunchKernelGGL(k_hist_lds, dim3((unsigned)g), dim3(256), 0, st, idx, n, (int)rows, bits, cnt);
    } else {
        if (g > 4096) g = 4096;
        hipLaunchKernelGGL(k_hist, dim3((unsigned)g), dim3(256), 0, st, idx, n, bits, cnt);
    }
}

}  // namespace s3
