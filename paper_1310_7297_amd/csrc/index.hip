// Device-resident obstacle index: a uniform grid of vertical columns.
//
// Replaces the paper's disk-based R*-tree (Sec. III-B), whose purpose there
// is to fetch only the obstacles near the lines of sight.  Here every column
// lists the boxes whose footprint, grown by kFatMargin, overlaps it; each
// list is sorted by decreasing top height so a ray that passes above a box
// can stop scanning the column there.  Built once per scene and kept in HBM
// (a few MB even for 100k boxes, so it lives in L2 during traversal).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "vcm_internal.h"

namespace vcm {
namespace {

struct BuildGrid {
    float fx, fy, fz;  // frame origin (boxes are stored relative to it)
    float inv_cs;
    int32_t nx, ny;
};

__device__ inline void footprint_cols(float lo, float hi, float org, float inv_cs, int32_t n,
                                      int32_t &a, int32_t &b) {
    // lo - margin and hi + margin are exact (multiples of 2^-8), and so is the
    // scaling by the power-of-two inverse cell size.
    a = static_cast<int32_t>(floorf((lo - kFatMargin - org) * inv_cs));
    b = static_cast<int32_t>(floorf((hi + kFatMargin - org) * inv_cs));
    a = max(0, min(n - 1, a));
    b = max(0, min(n - 1, b));
}

__global__ void k_count(const float *__restrict__ lo, const float *__restrict__ hi, int64_t n,
                        BuildGrid g, int32_t *__restrict__ counts) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t ax, bx, ay, by;
    footprint_cols(lo[i] - g.fx, hi[i] - g.fx, 0.0f, g.inv_cs, g.nx, ax, bx);
    footprint_cols(lo[n + i] - g.fy, hi[n + i] - g.fy, 0.0f, g.inv_cs, g.ny, ay, by);
    for (int32_t y = ay; y <= by; ++y)
        for (int32_t x = ax; x <= bx; ++x) atomicAdd(&counts[y * g.nx + x], 1);
}

// Exclusive scan of the list lengths (count + 1 for the sentinel that ends
// every column) into out[0..n], in three passes so that any number of columns
// spreads over the chip: each workgroup scans a tile of kScanTile columns and
// leaves the tile's total; one workgroup scans the totals; every tile then
// adds its offset.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;

// Exclusive scan of one value per thread across a workgroup of kScanThreads;
// returns the workgroup's total.
__device__ inline int32_t block_exclusive_scan(int32_t &v, int32_t *part) {
    const int t = threadIdx.x;
    part[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int32_t a = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += a;
        __syncthreads();
    }
    const int32_t total = part[kScanThreads - 1];
    v = part[t] - v;
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int32_t *__restrict__ counts, int32_t n,
                                                             int32_t *__restrict__ out,
                                                             int32_t *__restrict__ tile_sums) {
    __shared__ int32_t part[kScanThreads];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanPer;
    int32_t v[kScanPer], s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < n ? counts[base + k] + 1 : 0;
        s += v[k];
    }
    const int32_t total = block_exclusive_scan(s, part);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) out[base + k] = s;
        s += v[k];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the tile totals in place, the grand total
// into out[n].
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(int32_t *__restrict__ tile_sums, int32_t tiles,
                                                              int32_t *__restrict__ out, int32_t n) {
    __shared__ int32_t part[kScanThreads];
    int32_t carry = 0;
    for (int32_t b = 0; b < tiles; b += kScanThreads) {
        const int32_t i = b + threadIdx.x;
        int32_t v = i < tiles ? tile_sums[i] : 0;
        const int32_t total = block_exclusive_scan(v, part);
        if (i < tiles) tile_sums[i] = v + carry;
        carry += total;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(const int32_t *__restrict__ tile_sums, int32_t n,
                                                           int32_t *__restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x;
    const int32_t add = tile_sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (i + k * kScanThreads < n) out[i + k * kScanThreads] += add;
}

// Sort key of a record: decreasing top height, then increasing box id.  Tops
// are >= 0 in the index frame (or +inf), so their bit patterns order as
// unsigned integers.
__device__ inline uint64_t sort_key(float top, int32_t id) {
    return (static_cast<uint64_t>(~__float_as_uint(top)) << 32) | static_cast<uint32_t>(id);
}

__global__ void k_fill(const float *__restrict__ lo, const float *__restrict__ hi, int64_t n,
                       int32_t dim, BuildGrid g, int32_t *__restrict__ cursor,
                       BoxRec *__restrict__ recs, uint64_t *__restrict__ keys) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    BoxRec r;
    const float f[3] = {g.fx, g.fy, g.fz};
    for (int k = 0; k < 3; ++k) {
        // exact: both terms are multiples of 2^-8 and the result is below 2^15
        r.lo[k] = (k < dim) ? lo[k * n + i] - f[k] : 0.0f;
        r.hi[k] = (k < dim) ? hi[k * n + i] - f[k] : INFINITY;
    }
    r.id = static_cast<int32_t>(i);
    r.pad = 0;
    const uint64_t key = sort_key(r.hi[2], r.id);
    int32_t ax, bx, ay, by;
    footprint_cols(r.lo[0], r.hi[0], 0.0f, g.inv_cs, g.nx, ax, bx);
    footprint_cols(r.lo[1], r.hi[1], 0.0f, g.inv_cs, g.ny, ay, by);
    for (int32_t y = ay; y <= by; ++y)
        for (int32_t x = ax; x <= bx; ++x) {
            int32_t slot = atomicAdd(&cursor[y * g.nx + x], 1);
            recs[slot] = r;
            keys[slot] = key;
        }
}

// Sort every column list by (top height descending, box id ascending), which
// also makes the index independent of the order the atomics handed out
// slots, and end it with the sentinel: a record whose top is -inf, bit
// pattern 0xff800000, so that its difference with any floor of the traversal
// (an ordered integer in [0, 0x7f800000]) is negative as a signed integer,
// and whose lower corner is +inf.
//
// One thread per slot of the filled lists: it finds its column by binary
// search over the list starts and moves its record to the rank of its key
// among the column's keys (keys are distinct, so the ranks are a
// permutation).  A column of n records costs n key reads per record, all
// columns in parallel; neighbouring threads of one column read the same key
// at the same time.
__global__ __launch_bounds__(256) void k_rank(const int32_t *__restrict__ col_start, int32_t ncols,
                                              const BoxRec *__restrict__ in, const uint64_t *__restrict__ keys,
                                              int32_t total, BoxRec *__restrict__ out) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= total) return;
    int32_t a = 0, b = ncols;  // col_start[a] <= p < col_start[b]
    while (b - a > 1) {
        const int32_t m = (a + b) >> 1;
        if (col_start[m] <= p) a = m;
        else b = m;
    }
    const int32_t cb = col_start[a], ce = col_start[a + 1] - 1;  // ce: the sentinel's slot
    if (p == ce) {
        BoxRec sen;
        for (int k = 0; k < 3; ++k) {
            sen.lo[k] = INFINITY;
            sen.hi[k] = -INFINITY;
        }
        sen.id = -1;
        sen.pad = 0;
        out[p] = sen;
        return;
    }
    const uint64_t key = keys[p];
    int32_t rank = 0;
    for (int32_t j = cb; j < ce; ++j) rank += keys[j] < key;
    out[cb + rank] = in[p];
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return set_error(e_ == hipErrorOutOfMemory ? VCM_E_NOMEM : VCM_E_DEVICE,        \
                             std::string(#expr) + ": " + hipGetErrorString(e_));            \
    } while (0)

}  // namespace

vcm_status build_index_device(Index *ix, const float *h_lo, const float *h_hi, int64_t n,
                              double cell_size, hipStream_t stream) {
    auto t0 = std::chrono::steady_clock::now();
    // Column grid over the grown footprints.
    double mnx = 0, mny = 0, mxx = 0, mxy = 0, mnz = 0;
    if (n > 0) {
        mnx = mny = 1e30;
        mxx = mxy = -1e30;
        for (int64_t i = 0; i < n; ++i) {
            mnx = std::min(mnx, (double)h_lo[i]);
            mny = std::min(mny, (double)h_lo[n + i]);
            mxx = std::max(mxx, (double)h_hi[i]);
            mxy = std::max(mxy, (double)h_hi[n + i]);
            if (ix->dim == 3) mnz = std::min(mnz, (double)h_lo[2 * n + i]);
        }
    }
    double cs = cell_size;
    if (cs <= 0) {
        double area = std::max(1.0, (mxx - mnx) * (mxy - mny));
        double side = std::sqrt(area / std::max<int64_t>(n, 1));
        cs = std::ldexp(1.0, (int)std::lround(std::log2(std::max(side, 1.0))));
        cs = std::min(std::max(cs, 1.0), 1024.0);
    }
    int e2;
    if (std::frexp(cs, &e2) != 0.5 || cs < 1.0 / 16 || cs > 4096)
        return set_error(VCM_E_INVALID, "cell_size must be a power of two in [1/16, 4096]");
    double x0 = std::floor((mnx - kFatMargin) / cs) * cs;
    double y0 = std::floor((mny - kFatMargin) / cs) * cs;
    int64_t nx = (int64_t)std::floor((mxx + kFatMargin - x0) / cs) + 1;
    int64_t ny = (int64_t)std::floor((mxy + kFatMargin - y0) / cs) + 1;
    // at most 2^24 columns, and at most 65535 along each axis (the traversal
    // packs two column indices into one 32-bit word)
    while (nx * ny > (int64_t(1) << 24) || nx > 65535 || ny > 65535) {
        cs *= 2;
        x0 = std::floor((mnx - kFatMargin) / cs) * cs;
        y0 = std::floor((mny - kFatMargin) / cs) * cs;
        nx = (int64_t)std::floor((mxx + kFatMargin - x0) / cs) + 1;
        ny = (int64_t)std::floor((mxy + kFatMargin - y0) / cs) + 1;
    }
    const int32_t ncols = (int32_t)(nx * ny);
    BuildGrid g{(float)x0, (float)y0, (float)mnz, (float)(1.0 / cs), (int32_t)nx, (int32_t)ny};

    float *d_lo = nullptr, *d_hi = nullptr;
    int32_t *d_counts = nullptr, *d_cursor = nullptr, *d_tiles = nullptr;
    BoxRec *d_tmp = nullptr;
    uint64_t *d_keys = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // every exit frees what the build allocated for itself
    struct Cleanup {
        float *&lo, *&hi;
        int32_t *&counts, *&cursor, *&tiles;
        BoxRec *&tmp;
        uint64_t *&keys;
        hipEvent_t *ev;
        ~Cleanup() {
            if (lo) hipFree(lo);
            if (hi) hipFree(hi);
            if (counts) hipFree(counts);
            if (cursor) hipFree(cursor);
            if (tiles) hipFree(tiles);
            if (tmp) hipFree(tmp);
            if (keys) hipFree(keys);
            for (int k = 0; k < 4; ++k)
                if (ev[k]) hipEventDestroy(ev[k]);
        }
    } cleanup{d_lo, d_hi, d_counts, d_cursor, d_tiles, d_tmp, d_keys, ev};
    const size_t nb = (size_t)std::max<int64_t>(n, 1) * 3 * sizeof(float);
    const int32_t tiles = (ncols + kScanTile - 1) / kScanTile;
    HIP_TRY(hipMalloc(&d_lo, nb));
    HIP_TRY(hipMalloc(&d_hi, nb));
    HIP_TRY(hipMalloc(&d_counts, sizeof(int32_t) * ncols));
    HIP_TRY(hipMalloc(&d_tiles, sizeof(int32_t) * tiles));
    HIP_TRY(hipMalloc(&ix->d_col_start, sizeof(int32_t) * (ncols + 1)));
    HIP_TRY(hipMalloc(&d_cursor, sizeof(int32_t) * ncols));
    for (int k = 0; k < 4; ++k) HIP_TRY(hipEventCreate(&ev[k]));
    if (n > 0) {
        HIP_TRY(hipMemcpyAsync(d_lo, h_lo, sizeof(float) * 3 * n, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipMemcpyAsync(d_hi, h_hi, sizeof(float) * 3 * n, hipMemcpyHostToDevice, stream));
    }
    HIP_TRY(hipMemsetAsync(d_counts, 0, sizeof(int32_t) * ncols, stream));
    HIP_TRY(hipEventRecord(ev[0], stream));
    const int T = 256;
    if (n > 0)
        hipLaunchKernelGGL(k_count, dim3((unsigned)((n + T - 1) / T)), dim3(T), 0, stream, d_lo,
                           d_hi, n, g, d_counts);
    hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kScanThreads), 0, stream, d_counts, ncols,
                       ix->d_col_start, d_tiles);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, stream, d_tiles, tiles,
                       ix->d_col_start, ncols);
    hipLaunchKernelGGL(k_scan_add, dim3(tiles), dim3(kScanThreads), 0, stream, d_tiles, ncols,
                       ix->d_col_start);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(ev[1], stream));
    int32_t total = 0;
    HIP_TRY(hipMemcpyAsync(&total, ix->d_col_start + ncols, sizeof(int32_t),
                           hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipMalloc(&ix->d_recs, sizeof(BoxRec) * std::max(total, 1)));
    HIP_TRY(hipMalloc(&d_tmp, sizeof(BoxRec) * std::max(total, 1)));
    HIP_TRY(hipMalloc(&d_keys, sizeof(uint64_t) * std::max(total, 1)));
    BoxRec *d_recs = ix->d_recs;
    HIP_TRY(hipEventRecord(ev[2], stream));
    HIP_TRY(hipMemcpyAsync(d_cursor, ix->d_col_start, sizeof(int32_t) * ncols,
                           hipMemcpyDeviceToDevice, stream));
    if (n > 0)
        hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + T - 1) / T)), dim3(T), 0, stream, d_lo,
                           d_hi, n, ix->dim, g, d_cursor, d_tmp, d_keys);
    hipLaunchKernelGGL(k_rank, dim3((unsigned)((total + T - 1) / T)), dim3(T), 0, stream,
                       ix->d_col_start, ncols, d_tmp, d_keys, total, d_recs);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(ev[3], stream));
    HIP_TRY(hipStreamSynchronize(stream));
    // device time of the build kernels (the host's wait for the list total
    // between the two halves is not counted)
    float ms_a = 0.0f, ms_b = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms_a, ev[0], ev[1]));
    HIP_TRY(hipEventElapsedTime(&ms_b, ev[2], ev[3]));
    const double all_ms = static_cast<double>(ms_a) + ms_b;
    // host copy of the lists, for argument checks that need the obstacles
    ix->h_col_start.resize(static_cast<size_t>(ncols) + 1);
    ix->h_recs.resize(static_cast<size_t>(std::max(total, 1)));
    HIP_TRY(hipMemcpy(ix->h_col_start.data(), ix->d_col_start, sizeof(int32_t) * (ncols + 1),
                      hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ix->h_recs.data(), d_recs, sizeof(BoxRec) * std::max(total, 1), hipMemcpyDeviceToHost));
    int32_t longest = 0;
    for (int32_t c = 0; c < ncols; ++c)
        longest = std::max(longest, ix->h_col_start[c + 1] - ix->h_col_start[c] - 1);

    ix->n_boxes = n;
    ix->n_refs = total - ncols;  // without the sentinels
    ix->dev.col_start = ix->d_col_start;
    ix->dev.recs = ix->d_recs;
    ix->frame[0] = x0;
    ix->frame[1] = y0;
    ix->frame[2] = ix->dim == 3 ? mnz : 0.0;
    ix->dev.x0 = 0.0f;
    ix->dev.y0 = 0.0f;
    ix->dev.cs = (float)cs;
    ix->dev.inv_cs = (float)(1.0 / cs);
    ix->dev.nx = (int32_t)nx;
    ix->dev.ny = (int32_t)ny;
    ix->dev.dim = ix->dim;
    ix->bytes = sizeof(int32_t) * (ncols + 1) + sizeof(BoxRec) * std::max(total, 1);
    ix->longest_list = longest;
    ix->build_kernel_ms = all_ms;
    ix->build_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return VCM_OK;
}

}  // namespace vcm
