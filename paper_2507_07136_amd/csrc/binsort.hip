// ls2_bin_sort: (tile, Gaussian) pairs grouped by tile and ordered by
// (float32 depth, id) inside each tile -- the "ordered Gaussian points within
// a tile" that Eq. 3 composites.
//
// Pipeline (all on `stream`):
//   1. k_count   : per Gaussian, +1/-1 at the four corners of its tile
//                  rectangle in a (ty+1) x (tx+1) difference grid (4 atomics
//                  per Gaussian instead of one per touched tile).
//   2. k_scan    : one workgroup: 2D prefix sums turn the difference grid into
//                  per-tile counts, then an exclusive scan gives tile ranges
//                  and per-tile cursors, and the pair total P.
//   3. k_emit    : per Gaussian, claim a slot in each touched tile's bucket and
//                  store the 64-bit sort key (depth bits << 32 | id).
//   4. k_sort_*  : one workgroup per tile sorts its bucket in LDS (bitonic
//                  network over unique 64-bit keys, so the order is exact and
//                  independent of the emit order) and writes ids / keys.
#include "ls2_internal.h"

namespace ls2 {

namespace {

struct Meta {
    long long P;          // total pairs
    long long overflow;   // 1 if P > max_pairs
};

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
    size_t meta, grid, cursor, bucket, total;
};

inline Layout layout(const CamK& k, int64_t max_pairs) {
    Layout l;
    size_t off = 0;
    l.meta = off; off = align_up(off + sizeof(Meta));
    l.grid = off; off = align_up(off + sizeof(int) * (size_t)(k.tx + 1) * (k.ty + 1));
    l.cursor = off; off = align_up(off + sizeof(unsigned) * (size_t)k.tx * k.ty);
    l.bucket = off; off = align_up(off + sizeof(unsigned long long) * (size_t)(max_pairs > 0 ? max_pairs : 1));
    l.total = off;
    return l;
}

}  // namespace

__global__ void k_fill_zero(int* __restrict__ p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ __launch_bounds__(256) void k_count(CamK cam, int n, const float* __restrict__ mean2d,
                                               const int* __restrict__ radius, int* __restrict__ grid) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = radius[i];
    if (r <= 0) return;
    const float2 m = reinterpret_cast<const float2*>(mean2d)[i];
    int x0, y0, x1, y1;
    if (!tile_rect(m.x, m.y, r, cam.tx, cam.ty, x0, y0, x1, y1)) return;
    const int w = cam.tx + 1;
    atomicAdd(&grid[y0 * w + x0], 1);
    atomicAdd(&grid[y0 * w + x1 + 1], -1);
    atomicAdd(&grid[(y1 + 1) * w + x0], -1);
    atomicAdd(&grid[(y1 + 1) * w + x1 + 1], 1);
}

// Single workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan(CamK cam, int* __restrict__ grid, unsigned* __restrict__ cursor,
                                               unsigned* __restrict__ ranges, Meta* __restrict__ meta,
                                               long long max_pairs) {
    const int tid = threadIdx.x;
    const int w = cam.tx + 1;
    // row prefix sums
    for (int y = tid; y < cam.ty; y += blockDim.x) {
        int s = 0;
        for (int x = 0; x < cam.tx; ++x) {
            s += grid[y * w + x];
            grid[y * w + x] = s;
        }
    }
    __syncthreads();
    // column prefix sums -> per-tile counts
    for (int x = tid; x < cam.tx; x += blockDim.x) {
        int s = 0;
        for (int y = 0; y < cam.ty; ++y) {
            s += grid[y * w + x];
            grid[y * w + x] = s;
        }
    }
    __syncthreads();
    // exclusive scan over tiles (row-major), 1024 at a time
    __shared__ long long part[1024];
    __shared__ long long carry_s;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    const int ntiles = cam.tx * cam.ty;
    for (int base = 0; base < ntiles; base += 1024) {
        const int t = base + tid;
        long long c = 0;
        if (t < ntiles) c = grid[(t / cam.tx) * w + (t % cam.tx)];
        part[tid] = c;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            long long v = tid >= off ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += v;
            __syncthreads();
        }
        const long long incl = part[tid] + carry_s;
        if (t < ntiles) {
            // provisional: start in ranges[2t], count in ranges[2t+1]
            ranges[2 * t] = (unsigned)(incl - c);
            ranges[2 * t + 1] = (unsigned)c;
        }
        __syncthreads();
        if (tid == 1023) carry_s = incl;
        __syncthreads();
    }
    const long long P = carry_s;
    const bool overflow = P > max_pairs;
    for (int t = tid; t < ntiles; t += blockDim.x) {
        const unsigned start = ranges[2 * t], cnt = ranges[2 * t + 1];
        if (overflow) {
            ranges[2 * t] = 0;
            ranges[2 * t + 1] = 0;
        } else {
            ranges[2 * t + 1] = start + cnt;
            cursor[t] = start;
        }
    }
    if (tid == 0) {
        meta->P = P;
        meta->overflow = overflow ? 1 : 0;
    }
}

__global__ __launch_bounds__(256) void k_emit(CamK cam, int n, const float* __restrict__ mean2d,
                                              const int* __restrict__ radius, const float* __restrict__ depth,
                                              unsigned* __restrict__ cursor,
                                              unsigned long long* __restrict__ bucket,
                                              const Meta* __restrict__ meta) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (meta->overflow) return;
    const int r = radius[i];
    if (r <= 0) return;
    const float2 m = reinterpret_cast<const float2*>(mean2d)[i];
    int x0, y0, x1, y1;
    if (!tile_rect(m.x, m.y, r, cam.tx, cam.ty, x0, y0, x1, y1)) return;
    const unsigned long long key = ((unsigned long long)__float_as_uint(depth[i]) << 32) | (unsigned)i;
    for (int ty = y0; ty <= y1; ++ty)
        for (int tx = x0; tx <= x1; ++tx) {
            const unsigned pos = atomicAdd(&cursor[ty * cam.tx + tx], 1u);
            bucket[pos] = key;
        }
}

// Sorting network: bitonic sort in its all-ascending ("flip") form.  Stage k
// first compares i with i ^ (k - 1) (which reverses the upper half of every
// k-block), then runs half-cleaners i ^ j for j = k/4 .. 1; every comparator
// puts the smaller key at the lower index.  Because of that, padding the
// input to a power of two with +infinity keys is equivalent to skipping every
// comparator whose partner lies at or beyond `cnt`: such a comparator would
// never move anything.  No padding is stored.

// One tile's keys in LDS.  Handles tiles with lo < count <= CAP.
template <int CAP, int THREADS>
__global__ __launch_bounds__(THREADS) void k_sort_lds(int ntiles, const unsigned* __restrict__ ranges,
                                                      const unsigned long long* __restrict__ bucket,
                                                      unsigned* __restrict__ ids,
                                                      unsigned long long* __restrict__ keys, int lo) {
    __shared__ unsigned long long s[CAP];
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const unsigned start = ranges[2 * t], end = ranges[2 * t + 1];
    const int cnt = (int)(end - start);
    if (cnt <= lo || cnt > CAP) return;
    int m = 1;
    while (m < cnt) m <<= 1;
    for (int i = threadIdx.x; i < cnt; i += THREADS) s[i] = bucket[start + i];
    __syncthreads();
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int mask = (j == (k >> 1)) ? (k - 1) : j;  // flip first, then half-cleaners
            for (int i = threadIdx.x; i < m; i += THREADS) {
                const int p = i ^ mask;
                if (p > i && p < cnt) {
                    const unsigned long long a = s[i], b = s[p];
                    if (a > b) {
                        s[i] = b;
                        s[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    const unsigned long long tk = (unsigned long long)t << 32;
    for (int i = threadIdx.x; i < cnt; i += THREADS) {
        const unsigned long long v = s[i];
        ids[start + i] = (unsigned)(v & 0xffffffffull);
        if (keys) keys[start + i] = tk | (v >> 32);
    }
}

// Tiles longer than the LDS capacity: the same network in global memory, in
// place in the bucket.
__global__ __launch_bounds__(1024) void k_sort_global(int ntiles, const unsigned* __restrict__ ranges,
                                                      unsigned long long* __restrict__ bucket,
                                                      unsigned* __restrict__ ids,
                                                      unsigned long long* __restrict__ keys, int lo) {
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const unsigned start = ranges[2 * t], end = ranges[2 * t + 1];
    const int cnt = (int)(end - start);
    if (cnt <= lo) return;
    unsigned long long* s = bucket + start;
    int m = 1;
    while (m < cnt) m <<= 1;
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int mask = (j == (k >> 1)) ? (k - 1) : j;
            for (int i = threadIdx.x; i < m; i += blockDim.x) {
                const int p = i ^ mask;
                if (p > i && p < cnt) {
                    const unsigned long long a = s[i], b = s[p];
                    if (a > b) {
                        s[i] = b;
                        s[p] = a;
                    }
                }
            }
            __threadfence_block();
            __syncthreads();
        }
    }
    const unsigned long long tk = (unsigned long long)t << 32;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const unsigned long long v = s[i];
        ids[start + i] = (unsigned)(v & 0xffffffffull);
        if (keys) keys[start + i] = tk | (v >> 32);
    }
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_bin_sort_workspace(const ls2_camera* cam, int32_t n, int64_t max_pairs, size_t* bytes) {
    if (!cam_valid(cam) || n < 0 || max_pairs < 0 || !bytes) return LS2_ERR_ARG;
    if (max_pairs > 0xffffffffll) return LS2_ERR_UNSUPPORTED;  // 32-bit list positions
    *bytes = layout(cam_k(*cam), max_pairs).total;
    return LS2_OK;
}

extern "C" int ls2_bin_sort(const ls2_camera* cam, int32_t n, const float* mean2d, const int32_t* radius,
                            const float* depth, int64_t max_pairs, uint64_t* keys, uint32_t* ids,
                            uint32_t* tile_ranges, int64_t* num_pairs, void* workspace, size_t workspace_bytes,
                            hipStream_t stream) {
    if (!cam_valid(cam) || n < 0 || max_pairs < 0 || !tile_ranges || !workspace) return LS2_ERR_ARG;
    if (n > 0 && (!mean2d || !radius || !depth)) return LS2_ERR_ARG;
    if (max_pairs > 0 && !ids) return LS2_ERR_ARG;
    if (max_pairs > 0xffffffffll) return LS2_ERR_UNSUPPORTED;
    if (((uintptr_t)workspace & (kAlign - 1)) != 0) return LS2_ERR_ARG;
    const CamK k = cam_k(*cam);
    const Layout lay = layout(k, max_pairs);
    if (workspace_bytes < lay.total) return LS2_ERR_ARG;
    char* ws = static_cast<char*>(workspace);
    Meta* meta = reinterpret_cast<Meta*>(ws + lay.meta);
    int* grid = reinterpret_cast<int*>(ws + lay.grid);
    unsigned* cursor = reinterpret_cast<unsigned*>(ws + lay.cursor);
    unsigned long long* bucket = reinterpret_cast<unsigned long long*>(ws + lay.bucket);
    const int ntiles = k.tx * k.ty;

    // zero the meta record and the difference grid (contiguous)
    const long long zero_words = (long long)((lay.cursor - lay.meta) / sizeof(int));
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((zero_words + 255) / 256 < 1024 ? (zero_words + 255) / 256 : 1024)),
                       dim3(256), 0, stream, reinterpret_cast<int*>(ws + lay.meta), zero_words);
    LS2_LAUNCH_CHECK();
    if (n > 0) {
        hipLaunchKernelGGL(k_count, dim3((n + 255) / 256), dim3(256), 0, stream, k, n, mean2d, radius, grid);
        LS2_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, stream, k, grid, cursor, tile_ranges, meta,
                       (long long)max_pairs);
    LS2_LAUNCH_CHECK();
    if (n > 0 && max_pairs > 0) {
        hipLaunchKernelGGL(k_emit, dim3((n + 255) / 256), dim3(256), 0, stream, k, n, mean2d, radius, depth, cursor,
                           bucket, meta);
        LS2_LAUNCH_CHECK();
        unsigned long long* keys64 = reinterpret_cast<unsigned long long*>(keys);
        hipLaunchKernelGGL((k_sort_lds<512, 256>), dim3(ntiles), dim3(256), 0, stream, ntiles, tile_ranges, bucket,
                           ids, keys64, 0);
        LS2_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_sort_lds<2048, 512>), dim3(ntiles), dim3(512), 0, stream, ntiles, tile_ranges, bucket,
                           ids, keys64, 512);
        LS2_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_sort_lds<16384, 1024>), dim3(ntiles), dim3(1024), 0, stream, ntiles, tile_ranges,
                           bucket, ids, keys64, 2048);
        LS2_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sort_global, dim3(ntiles), dim3(1024), 0, stream, ntiles, tile_ranges, bucket, ids,
                           keys64, 16384);
        LS2_LAUNCH_CHECK();
    }
    if (num_pairs) {
        Meta h;
        if (hipMemcpyAsync(&h, meta, sizeof(Meta), hipMemcpyDeviceToHost, stream) != hipSuccess) return LS2_ERR_DEVICE;
        if (hipStreamSynchronize(stream) != hipSuccess) return LS2_ERR_DEVICE;
        *num_pairs = h.P;
        if (h.overflow) return LS2_ERR_CAPACITY;
    }
    return LS2_OK;
}

extern "C" int ls2_bin_sort_count(const void* workspace, int64_t* num_pairs, hipStream_t stream) {
    if (!workspace || !num_pairs) return LS2_ERR_ARG;
    Meta h;
    if (hipMemcpyAsync(&h, workspace, sizeof(Meta), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return LS2_ERR_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return LS2_ERR_DEVICE;
    *num_pairs = h.P;
    return LS2_OK;
}
