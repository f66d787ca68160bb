// ls2_bin_sort: (tile, Gaussian) pairs grouped by tile and ordered by
// (float32 depth, id) inside each tile: the front-to-back order in which
// Eq. 3 composites a tile's Gaussians.
//
// The P (tile, Gaussian) pairs (about 33 per Gaussian at 1440x1080) are never
// sorted or counted with atomics one by one.  The work is done on
// superblocks of S x S tiles (S = 4: 64 x 64 pixels), which a Gaussian touches
// only 1-4 of, and the lists are laid out superblock by superblock
// (superblocks row-major, tiles row-major inside each), so that every
// superblock's list positions are known before its bucket is sorted:
//   1. k_sb_count : per Gaussian, its tile rectangle (stored as 4 x u16), +1
//                   for every superblock it touches and the number of its
//                   tiles inside that superblock, aggregated per workgroup in
//                   LDS histograms (one global atomic per workgroup and
//                   superblock); also the exact pair count P;
//   2. k_sb_emit  : every workgroup first scans the superblock entry counts
//                   into bucket offsets (in LDS; the first workgroup also
//                   writes the list offsets, the overflow decision and the
//                   processing order for pass 3), then puts each Gaussian's
//                   64-bit key (depth bits << 32 | id) into each touched
//                   superblock's bucket (LDS histogram again, one reserving
//                   atomic per workgroup and superblock, LDS cursors);
//   3. k_sb_sort  : one workgroup per superblock sorts its bucket in LDS
//                   (keys binned over the bucket's depth range, each key of
//                   a short bin placed by its rank, long bins by a bitonic network;
//                   buckets beyond the LDS capacity are first split into 256
//                   bins over their depth range, and runs of bins are sorted
//                   in LDS; only a single over-full bin falls back to a
//                   bitonic network in global memory), then writes its tiles'
//                   ranges and lists: each tile's list is the ordered
//                   subsequence of the sorted bucket whose rectangles cover
//                   the tile, an order-preserving ballot compaction, so every
//                   list comes out already in (depth, id) order.
#include "project_common.h"

namespace ls2 {

namespace {

struct Meta {
    long long P;            // total (tile, Gaussian) pairs
    long long overflow;     // 1 if P > max_pairs
    long long sb_total;     // total (superblock, Gaussian) entries
    long long sb_overflow;  // 1 if sb_total > max_pairs
    unsigned long long P_rect;  // sum of tile-rectangle areas (= P), from pass 1
    long long pad[3];
};

constexpr size_t kAlign = 256;
constexpr int kMaxSB = 4096;  // superblocks held in an LDS histogram
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Geo {
    int S, sbx, sby, nsb;
};

// Superblock edge (in tiles): the smallest power of two >= 4 that keeps the
// superblock count within the LDS histogram.
inline Geo geo(const CamK& k) {
    Geo g;
    g.S = 4;
    while (((k.tx + g.S - 1) / g.S) * ((k.ty + g.S - 1) / g.S) > kMaxSB) g.S *= 2;
    g.sbx = (k.tx + g.S - 1) / g.S;
    g.sby = (k.ty + g.S - 1) / g.S;
    g.nsb = g.sbx * g.sby;
    return g;
}

struct Layout {
    size_t meta, sb_count, sb_pairs, sb_cursor, sb_start, sb_pstart, sb_order, rect, pool, cov, total;
};

// meta, sb_count, sb_pairs and sb_cursor come first: they are zeroed every call.
inline Layout layout(const CamK& k, int n, int64_t max_pairs) {
    const Geo g = geo(k);
    Layout l;
    size_t off = 0;
    l.meta = off; off = align_up(off + sizeof(Meta));
    l.sb_count = off; off = align_up(off + sizeof(unsigned) * (size_t)g.nsb);
    l.sb_pairs = off; off = align_up(off + sizeof(unsigned) * (size_t)g.nsb);
    l.sb_cursor = off; off = align_up(off + sizeof(unsigned) * (size_t)g.nsb);
    l.sb_start = off; off = align_up(off + sizeof(unsigned) * (size_t)g.nsb);
    l.sb_pstart = off; off = align_up(off + sizeof(unsigned) * (size_t)g.nsb);
    l.sb_order = off; off = align_up(off + sizeof(unsigned) * (size_t)g.nsb);
    l.rect = off; off = align_up(off + sizeof(ushort4) * (size_t)(n > 0 ? n : 1));
    l.pool = off; off = align_up(off + sizeof(unsigned long long) * (size_t)(max_pairs > 0 ? max_pairs : 1));
    l.cov = off; off = align_up(off + sizeof(unsigned short) * (size_t)(max_pairs > 0 ? max_pairs : 1));
    l.total = off;
    return l;
}

}  // namespace

// The projection's inputs and outputs when the count pass also projects
// (ls2_project_bin_sort); means is null otherwise.
struct ProjIO {
    const float* means;
    const float* scales;
    const float* quats;
    float* mean2d;
    float* conic;
    float* depth;
    int* radius;
    int* touched;
};

struct BinArgs {
    CamK cam;
    int n, S, sbx, nsb;
    long long max_pairs;
    const float* mean2d;
    const int* radius;
    const float* depth;
    Meta* meta;
    unsigned* sb_count;   // (superblock, Gaussian) entries of each superblock
    unsigned* sb_pairs;   // (tile, Gaussian) pairs inside each superblock
    unsigned* sb_start;   // bucket offset of each superblock in the pool
    unsigned* sb_pstart;  // first list position of each superblock's tiles
    unsigned* sb_cursor;  // entries reserved so far in each bucket
    unsigned* sb_order;  // superblocks by decreasing bucket size (size classes)
    ushort4* rect;
    unsigned long long* pool;
    unsigned short* cov;  // S = 4: each pool entry's coverage of its superblock's tiles (bit 4 y + x)
    unsigned* ranges;
    unsigned* ids;
    unsigned long long* keys;
    ProjIO pj;
};

// Orders this wave's earlier shared/global writes before its later reads.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void k_bin_zero(unsigned* __restrict__ p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Tile rectangle (x0, y0, x1, y1) of a Gaussian from its radius and mean,
// with the projection's rule; false (and an empty rectangle) if it covers no
// tile.
__device__ __forceinline__ bool gauss_rect(const BinArgs& a, int r, float2 m, int& x0, int& y0, int& x1, int& y1) {
    x0 = 0, y0 = 0, x1 = -1, y1 = -1;
    return r > 0 && tile_rect(m.x, m.y, r, a.cam.tx, a.cam.ty, x0, y0, x1, y1);
}

constexpr int kBinThreads = 1024;
constexpr int kBinPerThread = 2;  // Gaussians per thread in the histogram passes (147 workgroups at 300k)

// PROJ: each Gaussian is projected here first (the same instructions as
// ls2_project, whose outputs are written too) and its rectangle taken from
// the results in registers.
template <bool PROJ>
__global__ __launch_bounds__(kBinThreads) void k_sb_count(BinArgs a) {
    __shared__ unsigned hist[kMaxSB];
    __shared__ unsigned area[kMaxSB];
    __shared__ unsigned long long area_sum;
    for (int s = threadIdx.x; s < a.nsb; s += kBinThreads) hist[s] = area[s] = 0u;
    if (threadIdx.x == 0) area_sum = 0ull;
    __syncthreads();
    const int base = blockIdx.x * kBinThreads * kBinPerThread;
    const int S = a.S;
    const int sh = __builtin_ctz((unsigned)S);
    int rad[kBinPerThread];
    float2 mean[kBinPerThread];
    if constexpr (PROJ) {
#pragma unroll
        for (int q = 0; q < kBinPerThread; ++q) {
            const int i = base + q * kBinThreads + threadIdx.x;
            rad[q] = 0;
            mean[q] = make_float2(0.f, 0.f);
            if (i < a.n) {
                const ProjOut o = project_one(a.cam, a.pj.means, a.pj.scales, a.pj.quats, i);
                store_proj(o, i, a.pj.mean2d, a.pj.conic, a.pj.depth, a.pj.radius, a.pj.touched);
                rad[q] = o.r;
                mean[q] = make_float2(o.u, o.v);
            }
        }
    } else {
        // every global read at once (the mean is read whatever the radius)
#pragma unroll
        for (int q = 0; q < kBinPerThread; ++q) {
            const int i = base + q * kBinThreads + threadIdx.x;
            rad[q] = i < a.n ? a.radius[i] : 0;
            mean[q] = i < a.n ? reinterpret_cast<const float2*>(a.mean2d)[i] : make_float2(0.f, 0.f);
        }
    }
    unsigned long long my_area = 0;
#pragma unroll
    for (int q = 0; q < kBinPerThread; ++q) {
        const int i = base + q * kBinThreads + threadIdx.x;
        int x0, y0, x1, y1;
        const bool vis = gauss_rect(a, rad[q], mean[q], x0, y0, x1, y1);
        if (i < a.n)  // the rectangle for the later passes; culled: an empty one
            a.rect[i] = vis ? make_ushort4((unsigned short)x0, (unsigned short)y0, (unsigned short)x1,
                                           (unsigned short)y1)
                            : make_ushort4(0xffff, 0xffff, 0, 0);
        if (vis) {
            my_area += (unsigned long long)(x1 - x0 + 1) * (unsigned long long)(y1 - y0 + 1);
            for (int sy = y0 >> sh; sy <= (y1 >> sh); ++sy) {
                const int h = min(y1, sy * S + S - 1) - max(y0, sy * S) + 1;
                for (int sx = x0 >> sh; sx <= (x1 >> sh); ++sx) {
                    const int w = min(x1, sx * S + S - 1) - max(x0, sx * S) + 1;
                    atomicAdd(&hist[sy * a.sbx + sx], 1u);
                    atomicAdd(&area[sy * a.sbx + sx], (unsigned)(w * h));  // the pairs inside the superblock
                }
            }
        }
    }
    if (my_area) atomicAdd(&area_sum, my_area);
    __syncthreads();
    for (int s = threadIdx.x; s < a.nsb; s += kBinThreads) {
        if (hist[s]) {
            atomicAdd(&a.sb_count[s], hist[s]);
            atomicAdd(&a.sb_pairs[s], area[s]);  // exact whenever P fits the lists (P < 2^32)
        }
    }
    if (threadIdx.x == 0 && area_sum) atomicAdd(&a.meta->P_rect, area_sum);
}

// Exclusive scan over `n` counts by one workgroup of 1024 threads, 8192 at a
// time with a running carry.  Writes start (and, if `end` is non-null, end)
// offsets; returns the total.
__device__ long long block_scan(const unsigned* in, unsigned* start, int sstride, unsigned* end, int n) {
    // 1024 threads, 8 consecutive elements per thread per round: a serial scan
    // inside the thread, a shuffle scan across the wave, one LDS step across
    // the 16 waves
    constexpr int PER = 8;
    __shared__ long long wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    long long carry = 0;
    for (int base = 0; base < n; base += 1024 * PER) {
        const int t0 = base + tid * PER;
        unsigned v[PER];
        long long loc = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            v[k] = t0 + k < n ? in[t0 + k] : 0u;
            loc += v[k];
        }
        long long x = loc;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const long long y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        long long run = carry + x - loc, tot = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wave) run += wsum[w];
            tot += wsum[w];
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (t0 + k < n) {
                start[(size_t)(t0 + k) * sstride] = (unsigned)run;
                run += v[k];
                if (end) end[(size_t)(t0 + k) * sstride] = (unsigned)run;
            }
        }
        carry += tot;
        __syncthreads();  // wsum is rewritten by the next round
    }
    return carry;
}

// Size class of a bucket for the processing order: 256-entry steps up to
// 8192, then 1024-entry steps (class 63: 39936 and more).
__device__ __forceinline__ int size_class(unsigned c) {
    return c < 8192u ? (int)(c >> 8) : 32 + (int)min(31u, (c - 8192u) >> 10);
}

// The sort kernel's inputs, written by the emission pass's first workgroup
// (every workgroup of that pass forms the bucket offsets itself, in LDS):
// bucket and list offsets in global memory, the totals and the overflow
// decision, and the processing order.
__device__ void sort_plan(const BinArgs& a, const unsigned* start, long long total, long long P, bool over) {
    __shared__ unsigned cls[64];
    for (int s = threadIdx.x; s < a.nsb; s += blockDim.x) a.sb_start[s] = start[s];
    // P is exact in 64 bits; the per-superblock pair counts are exact whenever
    // P fits the lists, which is the only case in which their offsets are used
    block_scan(a.sb_pairs, a.sb_pstart, 1, nullptr, a.nsb);
    if (threadIdx.x == 0) {
        a.meta->sb_total = total;
        a.meta->sb_overflow = total > a.max_pairs ? 1 : 0;
        a.meta->P = P;
        a.meta->overflow = over ? 1 : 0;
    }
    // processing order of the per-superblock kernel: largest buckets first
    // (a counting sort on the size class; order inside a class is arbitrary),
    // so the long sorts start in the first dispatch round
    if (threadIdx.x < 64) cls[threadIdx.x] = 0u;
    __syncthreads();
    for (int s = threadIdx.x; s < a.nsb; s += blockDim.x) atomicAdd(&cls[size_class(a.sb_count[s])], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned off = 0u;
        for (int c = 63; c >= 0; --c) {
            const unsigned t = cls[c];
            cls[c] = off;
            off += t;
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < a.nsb; s += blockDim.x)
        a.sb_order[atomicAdd(&cls[size_class(a.sb_count[s])], 1u)] = (unsigned)s;
}

// Entries a workgroup of the emission pass stages in LDS (about 9500 at
// 1440x1080: 2048 Gaussians of 4.7 superblocks each); a workgroup with more
// writes them in place instead.
constexpr int kEmitCap = 10240;

__global__ __launch_bounds__(kBinThreads) void k_sb_emit(BinArgs a) {
    __shared__ unsigned hist[kMaxSB];
    __shared__ unsigned start[kMaxSB];
    // the workgroup's entries grouped by superblock, then copied out in runs
    __shared__ unsigned long long skey[kEmitCap];
    __shared__ unsigned short smask[kEmitCap];
    __shared__ unsigned short ssb[kEmitCap];
    const int base = blockIdx.x * kBinThreads * kBinPerThread;
    const int sh = __builtin_ctz((unsigned)a.S);
    // every global read at once: the tile rectangles stored by the count pass
    // (culled Gaussians have an empty one), the depths, the overflow flag
    ushort4 r[kBinPerThread];
    float dep[kBinPerThread];
#pragma unroll
    for (int q = 0; q < kBinPerThread; ++q) {
        const int i = base + q * kBinThreads + threadIdx.x;
        r[q] = i < a.n ? a.rect[i] : make_ushort4(0xffff, 0xffff, 0, 0);
        dep[q] = i < a.n ? a.depth[i] : 0.0f;
    }
    // the bucket offsets: an exclusive scan of the entry counts, in every
    // workgroup (the counts are complete: the count pass has finished)
    const long long total = block_scan(a.sb_count, start, 1, nullptr, a.nsb);
    const long long P = (long long)a.meta->P_rect;
    const bool over = P > a.max_pairs;  // sb_total <= P: covers the pool too
    if (blockIdx.x == 0) sort_plan(a, start, total, P, over);
    for (int s = threadIdx.x; s < a.nsb; s += kBinThreads) hist[s] = 0u;
    __syncthreads();
    if (over) return;  // the lists will not be filled (the same decision in every thread)
#pragma unroll
    for (int q = 0; q < kBinPerThread; ++q)
        if (r[q].x <= r[q].z)
            for (int sy = r[q].y >> sh; sy <= (r[q].w >> sh); ++sy)
                for (int sx = r[q].x >> sh; sx <= (r[q].z >> sh); ++sx) atomicAdd(&hist[sy * a.sbx + sx], 1u);
    __syncthreads();
    // reserve this workgroup's range in every touched bucket (start becomes
    // the range's first place), then the local places: an exclusive scan of
    // the counts (hist becomes the local cursor); start - local start maps a
    // local place to its place in the pool
    for (int s = threadIdx.x; s < a.nsb; s += kBinThreads)
        if (hist[s]) start[s] += atomicAdd(&a.sb_cursor[s], hist[s]);
    __syncthreads();
    const long long mine = block_scan(hist, hist, 1, nullptr, a.nsb);  // in place: each thread rewrites what it read
    const bool staged = mine <= kEmitCap;  // the same decision in every thread
    for (int s = threadIdx.x; s < a.nsb; s += kBinThreads) start[s] -= hist[s];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kBinPerThread; ++q) {
        if (r[q].x > r[q].z) continue;
        const int i = base + q * kBinThreads + threadIdx.x;
        const unsigned long long key = ((unsigned long long)__float_as_uint(dep[q]) << 32) | (unsigned)i;
        const int x0 = r[q].x, y0 = r[q].y, x1 = r[q].z, y1 = r[q].w;
        for (int sy = y0 >> sh; sy <= (y1 >> sh); ++sy)
            for (int sx = x0 >> sh; sx <= (x1 >> sh); ++sx) {
                const int s = sy * a.sbx + sx;
                const unsigned lp = atomicAdd(&hist[s], 1u);
                unsigned short mask = 0;
                if (a.S == 4) {  // the tiles of the superblock the rectangle covers
                    const int cx0 = max(x0 - 4 * sx, 0), cx1 = min(x1 - 4 * sx, 3);
                    const int cy0 = max(y0 - 4 * sy, 0), cy1 = min(y1 - 4 * sy, 3);
                    const unsigned cols = ((2u << cx1) - 1u) & ~((1u << cx0) - 1u);
                    const unsigned rows = 0x1111u & ((1u << (4 * cy1 + 4)) - 1u) & ~((1u << (4 * cy0)) - 1u);
                    mask = (unsigned short)(cols * rows);
                }
                if (staged) {
                    skey[lp] = key;
                    smask[lp] = mask;
                    ssb[lp] = (unsigned short)s;
                } else {
                    const unsigned pos = start[s] + lp;
                    a.pool[pos] = key;
                    if (a.S == 4) a.cov[pos] = mask;
                }
            }
    }
    if (!staged) return;
    __syncthreads();
    // copy-out: consecutive local places of one superblock are consecutive
    // places in the pool, so neighbouring lanes write neighbouring words
    for (int j = threadIdx.x; j < (int)mine; j += kBinThreads) {
        const unsigned pos = start[ssb[j]] + (unsigned)j;
        a.pool[pos] = skey[j];
        if (a.S == 4) a.cov[pos] = smask[j];
    }
}

// Sorting network: bitonic sort in its all-ascending ("flip") form.  Stage k
// first compares i with i ^ (k - 1) (which reverses the upper half of every
// k-block), then runs half-cleaners i ^ j for j = k/4 .. 1; every comparator
// puts the smaller key at the lower index.  Because of that, padding the
// input to a power of two with +infinity keys is equivalent to skipping every
// comparator whose partner lies at or beyond `cnt`: such a comparator would
// never move anything.  No padding is stored.
template <bool WAVE_LOCAL, typename Ptr>
__device__ void flip_bitonic(Ptr s, int cnt, unsigned short* pay = nullptr) {
    int m = 1;
    while (m < cnt) m <<= 1;
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int mask = (j == (k >> 1)) ? (k - 1) : j;
            // a comparator spanning less than 64 positions pairs two indices
            // handled by the same wave (each wave owns 64-aligned index blocks),
            // so in LDS only that wave's earlier writes must be visible; the
            // global-memory variant always uses workgroup barriers
            if (mask >= 64 || !WAVE_LOCAL) {
                __threadfence_block();
                __syncthreads();
            } else {
                wave_sync();
            }
            for (int i = threadIdx.x; i < m; i += blockDim.x) {
                const int p = i ^ mask;
                if (p > i && p < cnt) {
                    const unsigned long long x = s[i], y = s[p];
                    if (x > y) {
                        s[i] = y;
                        s[p] = x;
                        if (pay) {  // the payload moves with its key
                            const unsigned short t = pay[i];
                            pay[i] = pay[p];
                            pay[p] = t;
                        }
                    }
                }
            }
        }
    }
    __threadfence_block();
    __syncthreads();
}

constexpr int kMaxS2 = 32 * 32;  // tile counters per superblock (S <= 32)

// LDS sort of one bucket (or one chunk of a large bucket).  A key is
// (float32 depth bits << 32 | id); ids are unique inside a bucket, so the
// keys are too, and their order is total.
constexpr int kSortCap = 16384;
constexpr int kSortWaves = 16;

struct SortSmem {
    unsigned long long xbuf[kSortCap];
    unsigned ctr[kSortWaves][256];
    unsigned tcnt[kMaxS2];          // list fill: tile counts, then tile list starts
    unsigned bits[4];           // large buckets: OR and AND of the keys
    unsigned hmin, hmax;        // large buckets: range of the keys' depth halves
    unsigned chunk_start[257];  // large buckets: key offset of each chunk
    unsigned nchunks;
    unsigned wred[kSortWaves][4];  // per-wave key ranges
    unsigned wscan[kSortWaves];    // per-wave bin totals
    unsigned big[kMaxS2];           // long bins: start | count << 15; then tile list ends
    unsigned nbig;
    unsigned wcnt[kSortWaves][16];  // list fill: entries of each wave's slice per tile of a block
};

// Sort of one bucket (or one chunk of a large bucket) in LDS: cnt <=
// kSortCap unique keys from src into dst (may alias); the sorted keys are
// also left in sm.xbuf[0, cnt).
//
// The keys are distributed over nb bins (the power of two >= cnt, within
// [64, 4096]) by a bin number that is non-decreasing in the key: the key's
// depth half mapped linearly onto the bucket's depth range (if every depth is
// equal, its id half onto the id range).  Every key of a lower bin is then
// smaller than every key of a higher one.  A histogram and its scan give each
// bin its place, and the keys are scattered there.  A key of a short bin
// then goes to its bin's start plus the number of the bin's keys below it,
// comparing whole 64-bit keys, so ties of depth are ordered by id with no
// extra step.  Bins of more than kBinSortMax keys (depths clustered more
// tightly than the bin width) are instead sorted one after another by the
// whole workgroup with the bitonic network in LDS.
//
// Called by the whole workgroup; the caller orders earlier LDS use of sm
// before the call, and the call ends with an LDS barrier (the global writes
// to dst are not waited for).
constexpr int kBinSortMax = 16;

// A 16-bit payload per key (the coverage masks) rides along with the sort
// when the bucket leaves room in sm.xbuf: the sorted payload follows the cnt
// keys, and the payload in bucket order follows it (12 bytes per key).
constexpr int kPayCap = 10240;
__device__ __forceinline__ unsigned short* pay_sorted(SortSmem& sm, int cnt) {
    return reinterpret_cast<unsigned short*>(sm.xbuf + cnt);  // 8-byte aligned
}
static_assert(kPayCap * (sizeof(unsigned long long) + 2 * sizeof(unsigned short)) + 8 <= sizeof(SortSmem::xbuf),
              "keys, payloads and a 4-mask read past the sorted payload fit the key buffer");

template <int ITEMS>  // 64-key chunks per wave, at most: cnt <= 64 kSortWaves ITEMS
__device__ __forceinline__ void sort_lds_n(SortSmem& sm, const unsigned long long* src, unsigned long long* dst,
                                           int cnt, const unsigned short* pay_src) {
    constexpr int NW = kSortWaves;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nchunk = (cnt + 63) >> 6;
    const int cpw = (nchunk + NW - 1) / NW;
    const int c0 = w * cpw;
    const int mine = max(0, min(cpw, nchunk - c0));  // this wave's chunks (wave-uniform)
    int nb = 64;
    while (nb < cnt && nb < 4096) nb <<= 1;
    unsigned* const bins = &sm.ctr[0][0];  // NW * 256 = 4096 counters

    unsigned long long key[ITEMS];
    unsigned short pv[ITEMS];  // the payload of each key (pay_src given), loaded with it
    unsigned hlo = 0xffffffffu, hhi = 0u, ilo = 0xffffffffu, ihi = 0u;
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        key[c] = 0ull;
        pv[c] = 0;
        const int p = (c0 + c) * 64 + lane;
        if (c < mine && p < cnt) {
            key[c] = src[p];
            if (pay_src) pv[c] = pay_src[p];
            const unsigned h = (unsigned)(key[c] >> 32), id = (unsigned)key[c];
            hlo = min(hlo, h);
            hhi = max(hhi, h);
            ilo = min(ilo, id);
            ihi = max(ihi, id);
        }
    }
    for (int i = threadIdx.x; i < nb; i += blockDim.x) bins[i] = 0u;
    if (threadIdx.x == 0) sm.nbig = 0u;
    // payload (cnt <= kPayCap): moved with the keys, from registers
    unsigned short* const pay = pay_src ? pay_sorted(sm, cnt) : nullptr;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        hlo = min(hlo, (unsigned)__shfl_xor((int)hlo, off));
        hhi = max(hhi, (unsigned)__shfl_xor((int)hhi, off));
        ilo = min(ilo, (unsigned)__shfl_xor((int)ilo, off));
        ihi = max(ihi, (unsigned)__shfl_xor((int)ihi, off));
    }
    if (lane == 0) {
        sm.wred[w][0] = hlo;
        sm.wred[w][1] = hhi;
        sm.wred[w][2] = ilo;
        sm.wred[w][3] = ihi;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NW; ++v) {
        hlo = min(hlo, sm.wred[v][0]);
        hhi = max(hhi, sm.wred[v][1]);
        ilo = min(ilo, sm.wred[v][2]);
        ihi = max(ihi, sm.wred[v][3]);
    }
    // bin number: non-decreasing in the key (every conversion and the
    // product by a positive factor are monotone; the clamp absorbs rounding)
    const bool by_id = hlo == hhi;
    const unsigned vbase = by_id ? ilo : hlo;
    const float vscale = (float)nb / ((float)(by_id ? ihi - ilo : hhi - hlo) + 1.0f);
    auto bin_of = [=](unsigned long long k) -> unsigned {
        const unsigned v = by_id ? (unsigned)k : (unsigned)(k >> 32);
        return min((unsigned)(nb - 1), (unsigned)((float)(v - vbase) * vscale));
    };
    // 1. histogram
#pragma unroll
    for (int c = 0; c < ITEMS; ++c)
        if (c < mine && (c0 + c) * 64 + lane < cnt) atomicAdd(&bins[bin_of(key[c])], 1u);
    __syncthreads();
    // 2. exclusive scan of the bin counts: thread t owns bins [t per, t per + per)
    const int per = (nb + (int)blockDim.x - 1) / (int)blockDim.x;  // 1, 2 or 4
    unsigned bc[4], loc = 0u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = (int)threadIdx.x * per + q;
        bc[q] = (q < per && i < nb) ? bins[i] : 0u;
        loc += bc[q];
    }
    unsigned incl = loc;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == 63) sm.wscan[w] = incl;
    __syncthreads();
    unsigned run = incl - loc;
#pragma unroll
    for (int v = 0; v < NW; ++v)
        if (v < w) run += sm.wscan[v];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = (int)threadIdx.x * per + q;
        if (q < per && i < nb) bins[i] = run;  // this thread alone read bins[i] above
        if (bc[q] > (unsigned)kBinSortMax)     // at most cnt / (kBinSortMax + 1) < kMaxS2 such bins
            sm.big[atomicAdd(&sm.nbig, 1u)] = run | bc[q] << 15;
        run += bc[q];
    }
    __syncthreads();
    // 3. scatter: each key to the next free place of its bin (the counters
    // are now cursors)
#pragma unroll
    for (int c = 0; c < ITEMS; ++c)
        if (c < mine && (c0 + c) * 64 + lane < cnt) {
            const unsigned slot = atomicAdd(&bins[bin_of(key[c])], 1u);
            sm.xbuf[slot] = key[c];
            if (pay) pay[slot] = pv[c];
        }
    __syncthreads();
    // 4. a key of a short bin goes to its bin's start plus the number of the
    // bin's keys below it (the cursors now hold each bin's end).  The first
    // four places of the bin are read at once, so most keys need one LDS
    // round trip; every read is done before any key moves.
    unsigned fp[ITEMS];
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        fp[c] = 0xffffffffu;
        if (c < mine && (c0 + c) * 64 + lane < cnt) {
            const unsigned b = bin_of(key[c]);
            const int b0 = b ? (int)bins[b - 1] : 0, n = (int)bins[b] - b0;
            if (n <= kBinSortMax) {
                unsigned r = 0u;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const unsigned long long v = sm.xbuf[min(b0 + j, cnt - 1)];
                    r += (j < n && v < key[c]) ? 1u : 0u;
                }
                for (int j = 4; j < n; ++j) r += sm.xbuf[b0 + j] < key[c] ? 1u : 0u;
                fp[c] = (unsigned)b0 + r;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < ITEMS; ++c)
        if (fp[c] != 0xffffffffu) {
            sm.xbuf[fp[c]] = key[c];
            if (pay) pay[fp[c]] = pv[c];
        }
    // 5. long bins, one at a time, by the whole workgroup (each network ends
    // with a workgroup barrier; they touch disjoint ranges, none a short bin)
    const unsigned nbig = sm.nbig;  // stored before the last barrier
    for (unsigned k = 0; k < nbig; ++k) {
        const unsigned e = sm.big[k];
        flip_bitonic<true>(sm.xbuf + (e & 0x7fffu), (int)(e >> 15), pay ? pay + (e & 0x7fffu) : nullptr);
    }
    lds_barrier();
    if (dst)  // the sorted keys back to global memory (chunks of a split bucket)
        for (int p = threadIdx.x; p < cnt; p += blockDim.x) dst[p] = sm.xbuf[p];
}

// Buckets of up to 9 x 1024 keys (all but the largest) hold 9 keys per
// thread in registers instead of 16.
constexpr int kSortSmallItems = 9;
__device__ __forceinline__ void sort_lds(SortSmem& sm, const unsigned long long* src, unsigned long long* dst,
                                         int cnt, const unsigned short* pay_src = nullptr) {
    if (cnt <= 64 * kSortWaves * kSortSmallItems)
        sort_lds_n<kSortSmallItems>(sm, src, dst, cnt, pay_src);
    else
        sort_lds_n<kSortCap / (64 * kSortWaves)>(sm, src, dst, cnt, pay_src);
}

// A bucket beyond kSortCap keys: split into the scratch copy by a digit over
// its depth range and return the number of LDS-sized chunks (their key offsets
// in sm.chunk_start); 0 if it was sorted here instead, with the global bitonic
// network (no room for the scratch copy, or one digit bin beyond kSortCap).
__device__ __forceinline__ int split_bucket(const BinArgs& a, SortSmem& sm, unsigned long long* g, int cnt) {
    const long long total = a.meta->sb_total;
    if (2 * total > a.max_pairs) {  // no room for the scratch copy
        flip_bitonic<false>(g, cnt);
        return 0;
    }
    unsigned long long* tmp = a.pool + total + (g - a.pool);
    // varying bits of the bucket, and the range of its depth halves
    unsigned long long kor = 0ull, kand = ~0ull;
    unsigned hlo = 0xffffffffu, hhi = 0u;
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        const unsigned long long k = g[e];
        kor |= k;
        kand &= k;
        hlo = min(hlo, (unsigned)(k >> 32));
        hhi = max(hhi, (unsigned)(k >> 32));
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        kor |= __shfl_xor(kor, off);
        kand &= __shfl_xor(kand, off);
        hlo = min(hlo, (unsigned)__shfl_xor((int)hlo, off));
        hhi = max(hhi, (unsigned)__shfl_xor((int)hhi, off));
    }
    if (threadIdx.x < 4) sm.bits[threadIdx.x] = threadIdx.x < 2 ? 0u : ~0u;
    if (threadIdx.x == 0) {
        sm.hmin = 0xffffffffu;
        sm.hmax = 0u;
    }
    for (int i = threadIdx.x; i < 256; i += blockDim.x) sm.ctr[0][i] = 0u;
    __syncthreads();
    if (lane == 0) {
        atomicOr(&sm.bits[0], (unsigned)kor);
        atomicOr(&sm.bits[1], (unsigned)(kor >> 32));
        atomicAnd(&sm.bits[2], (unsigned)kand);
        atomicAnd(&sm.bits[3], (unsigned)(kand >> 32));
        atomicMin(&sm.hmin, hlo);
        atomicMax(&sm.hmax, hhi);
    }
    __syncthreads();
    const unsigned long long varying = (((unsigned long long)sm.bits[1] << 32) | sm.bits[0]) ^
                                       (((unsigned long long)sm.bits[3] << 32) | sm.bits[2]);
    const int top = varying ? 63 - __builtin_clzll(varying) : 0;
    // Split digit, non-decreasing in the key so that the digit bins are
    // consecutive key ranges.  With varying depths it spreads the depth
    // halves' range over 256 bins; a power-of-two window of the key bits
    // would mostly see the float exponent (e.g. depths 1.5..4.5 give three
    // values), leaving bins too full for the LDS sort.  If every depth is
    // equal, the top eight varying bits (of the id) instead.
    const unsigned hmin = sm.hmin, hrange = sm.hmax - sm.hmin;
    const float hscale = 256.0f / ((float)hrange + 1.0f);
    const int dshift = top >= 7 ? top - 7 : 0;
    auto split_digit = [=](unsigned long long k) -> unsigned {
        if (hrange == 0u) return (unsigned)(k >> dshift) & 0xffu;
        return min(255u, (unsigned)((float)((unsigned)(k >> 32) - hmin) * hscale));
    };
    // histogram of the split digit
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) atomicAdd(&sm.ctr[0][split_digit(g[e])], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        // digit offsets, and runs of consecutive digits of at most kSortCap keys
        unsigned off = 0u, run = 0u, nch = 0u;
        bool ok = true;
        for (int d = 0; d < 256; ++d) {
            const unsigned c = sm.ctr[0][d];
            if (c > (unsigned)kSortCap) ok = false;
            if (run > 0u && run + c > (unsigned)kSortCap) {  // at most 255 closes: chunk_start fits
                sm.chunk_start[nch++] = off - run;
                run = 0u;
            }
            sm.ctr[1][d] = off;  // scatter cursor
            off += c;
            run += c;
        }
        sm.chunk_start[nch++] = off - run;
        sm.chunk_start[nch] = off;
        sm.nchunks = ok ? nch : 0u;
    }
    __syncthreads();
    const int nch = (int)sm.nchunks;
    if (nch == 0) {  // one digit bin holds more keys than the LDS sort: global bitonic network
        flip_bitonic<false>(g, cnt);
        return 0;
    }
    // scatter into the scratch copy by split digit (order inside a bin is not
    // needed: every chunk is fully sorted next)
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        const unsigned long long k = g[e];
        tmp[atomicAdd(&sm.ctr[1][split_digit(k)], 1u)] = k;
    }
    __threadfence_block();
    __syncthreads();
    return nch;
}

// Tile lists of one superblock from its sorted bucket s[0, cnt) (in LDS or in
// global memory).  The superblock's pairs occupy [sb_pstart, sb_pstart +
// sb_pairs) of the lists, its tiles in row-major order inside it.  The
// superblock is taken as (S/4)^2 blocks of 4 x 4 tiles, and an entry's
// coverage of a block is a 16-bit mask (bit 4 y + x).  Wave w owns the slice
// [w len, (w + 1) len) of the bucket (len a multiple of 64).  In a block,
// lane t of every wave counts the slice's entries that cover tile t (one
// ballot per tile and 64 entries); the waves' counts give each wave its first
// place in every tile; a second pass emits the entries in bucket order (per
// tile one ballot, the lane's place among the covering lanes, one store), so
// every tile list is the ordered subsequence of the sorted bucket.
constexpr int kFillGroups = 4;  // 64-entry groups loaded at once

// Emits the entries [e0, e1) of a sorted bucket into the 16 tiles of one
// 4 x 4-tile block at (ox, oy): lane t of cur holds tile t's next place, lane
// t of end its list end.  Per tile and 64 entries: one ballot, the lane's
// rank among the covering lanes (mbcnt), one store.
template <bool KEYS, typename Cover>
__device__ __forceinline__ void emit_slice(const unsigned long long* s, const ushort4* __restrict__ rect,
                                           __attribute__((address_space(1))) unsigned* ids,
                                           unsigned long long* __restrict__ keys, int e0, int e1, unsigned& cur,
                                           unsigned end, int tiles_x, int ox, int oy, Cover cover_rect, int bx,
                                           int by) {
    const int lane = threadIdx.x & 63;
    for (int e = e0; e < e1; e += 64 * kFillGroups) {
        unsigned long long kk[kFillGroups];
        ushort4 r[kFillGroups];
        unsigned cv[kFillGroups];
#pragma unroll
        for (int q = 0; q < kFillGroups; ++q) kk[q] = s[min(e + 64 * q + lane, e1 - 1)];
#pragma unroll
        for (int q = 0; q < kFillGroups; ++q) r[q] = rect[(unsigned)(kk[q] & 0xffffffffull)];
#pragma unroll
        for (int q = 0; q < kFillGroups; ++q) cv[q] = e + 64 * q + lane < e1 ? cover_rect(r[q], bx, by) : 0u;
        // one tile at a time: its cursor and end are the only per-tile scalars live
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            unsigned out = (unsigned)__builtin_amdgcn_readlane((int)cur, t);
            const unsigned tend = (unsigned)__builtin_amdgcn_readlane((int)end, t);
            const unsigned long long tk = (unsigned long long)((oy + (t >> 2)) * tiles_x + ox + (t & 3)) << 32;
#pragma unroll
            for (int q = 0; q < kFillGroups; ++q) {
                const unsigned long long mask = __builtin_amdgcn_ballot_w64((cv[q] >> t) & 1u);
                const unsigned pos = out + __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
                if (((mask >> lane) & 1ull) && pos < tend) {  // the counts use the same test: pos < tend always
                    ids[pos] = (unsigned)(kk[q] & 0xffffffffull);
                    if (KEYS) keys[pos] = tk | (kk[q] >> 32);
                }
                out += (unsigned)__builtin_popcountll(mask);
            }
            if (lane == t) cur = out;
        }
    }
}

__device__ __forceinline__ void fill_sb_lists(const BinArgs& a, SortSmem& sm, int sb, unsigned pstart,
                                              const unsigned long long* s, int cnt) {
    const int S = a.S, nsub = S >> 2;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int tx0 = (sb % a.sbx) * S, ty0 = (sb / a.sbx) * S;
    const int len = (cnt + 64 * kSortWaves - 1) / (64 * kSortWaves) * 64;
    // the list base lives in vector registers (global address space): the
    // scalar file is full here, and a scalar copy would be reloaded from the
    // kernel arguments before every store
    __attribute__((address_space(1))) unsigned* ids = (__attribute__((address_space(1))) unsigned*)a.ids;
    asm volatile("" : "+v"(ids));
    unsigned long long* __restrict__ const keys = a.keys;
    const ushort4* __restrict__ const rect = a.rect;
    const int e0 = min(cnt, w * len), e1 = min(cnt, e0 + len);
    // coverage of the block at tile offset (bx, by) of the superblock
    // (branch-free: the covered columns' bits times one bit 4 y per covered
    // row y; bounds clamped to [0, 4] and [-1, 3], so an empty range gives 0)
    auto cover_rect = [&](const ushort4 r, int bx, int by) -> unsigned {
        const int ox = tx0 + bx, oy = ty0 + by;
        const int x0 = min(max((int)r.x - ox, 0), 4), x1 = max(min((int)r.z - ox, 3), -1);
        const int y0 = min(max((int)r.y - oy, 0), 4), y1 = max(min((int)r.w - oy, 3), -1);
        const unsigned cols = ((1u << (x1 + 1)) - 1u) & ~((1u << x0) - 1u);
        const unsigned rows = 0x1111u & ((1u << (4 * (y1 + 1))) - 1u) & ~((1u << (4 * y0)) - 1u);
        return cols * rows;
    };
    // entries of this wave's slice covering each tile of a block (lane t: tile t)
    auto count_block = [&](int bx, int by) -> unsigned {
        unsigned mine = 0u;
        for (int e = e0; e < e1; e += 64 * kFillGroups) {
            // every load issued at once (positions past the slice read its last entry)
            unsigned long long k[kFillGroups];
            ushort4 r[kFillGroups];
#pragma unroll
            for (int q = 0; q < kFillGroups; ++q) k[q] = s[min(e + 64 * q + lane, e1 - 1)];
#pragma unroll
            for (int q = 0; q < kFillGroups; ++q) r[q] = rect[(unsigned)(k[q] & 0xffffffffull)];
#pragma unroll
            for (int q = 0; q < kFillGroups; ++q) {
                const unsigned cv = e + 64 * q + lane < e1 ? cover_rect(r[q], bx, by) : 0u;
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const unsigned c = (unsigned)__builtin_popcountll(__builtin_amdgcn_ballot_w64((cv >> t) & 1u));
                    if (lane == t) mine += c;
                }
            }
        }
        return mine;
    };
    // 1. tile totals, row-major in the superblock
    for (int t = threadIdx.x; t < S * S; t += blockDim.x) sm.tcnt[t] = 0u;
    __syncthreads();
    for (int k = 0; k < nsub * nsub; ++k) {
        const int bx = (k % nsub) * 4, by = (k / nsub) * 4;
        const unsigned c = count_block(bx, by);
        if (nsub == 1 && lane < 16) sm.wcnt[w][lane] = c;
        if (lane < 16 && c) atomicAdd(&sm.tcnt[(by + (lane >> 2)) * S + bx + (lane & 3)], c);
    }
    __syncthreads();
    // 2. list start and end of every tile; the tile ranges
    if (w == 0) {
        const int nt = S * S, per = (nt + 63) / 64;  // at most 16
        unsigned loc = 0u;
        for (int q = 0; q < per; ++q)
            if (lane * per + q < nt) loc += sm.tcnt[lane * per + q];
        unsigned incl = loc;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        unsigned run = pstart + incl - loc;
        for (int q = 0; q < per; ++q) {
            const int t = lane * per + q;
            if (t >= nt) break;
            const unsigned c = sm.tcnt[t];
            sm.tcnt[t] = run;
            sm.big[t] = run + c;
            const int x = tx0 + t % S, y = ty0 + t / S;
            if (x < a.cam.tx && y < a.cam.ty) {
                a.ranges[2 * (y * a.cam.tx + x)] = run;
                a.ranges[2 * (y * a.cam.tx + x) + 1] = run + c;
            }
            run += c;
        }
    }
    __syncthreads();
    // 3. emit, block by block
    for (int k = 0; k < nsub * nsub; ++k) {
        const int bx = (k % nsub) * 4, by = (k / nsub) * 4;
        if (nsub > 1) {
            const unsigned c = count_block(bx, by);
            if (lane < 16) sm.wcnt[w][lane] = c;
            __syncthreads();
        }
        // lane t: this wave's next place in tile t of the block, and the tile's end
        unsigned cur = 0u, end = 0u;
        if (lane < 16) {
            const int t = (by + (lane >> 2)) * S + bx + (lane & 3);
            cur = sm.tcnt[t];
            for (int v = 0; v < w; ++v) cur += sm.wcnt[v][lane];
            end = min(sm.big[t], (unsigned)a.max_pairs);  // P <= max_pairs here; the clamp only guards
        }
        if (keys)
            emit_slice<true>(s, rect, ids, keys, e0, e1, cur, end, a.cam.tx, tx0 + bx, ty0 + by, cover_rect, bx, by);
        else
            emit_slice<false>(s, rect, ids, keys, e0, e1, cur, end, a.cam.tx, tx0 + bx, ty0 + by, cover_rect, bx, by);
        if (nsub > 1) __syncthreads();  // sm.wcnt is rewritten for the next block
    }
}

// Tile lists of a 4 x 4-tile superblock whose bucket (cnt <= kPayCap) was
// sorted in sm.xbuf together with its coverage masks (bit 4 y + x, written by
// k_sb_emit).  Wave w owns the slice [w len, (w + 1) len) of the bucket (len
// a multiple of 64): it counts the slice's entries per tile (one ballot per
// tile and 64 entries), the waves' counts give each wave its first place in
// every tile, and a second pass emits the slice in order (per tile one
// ballot, the lane's rank among the covering lanes, one store), so every
// tile list is the ordered subsequence of the sorted bucket.  Masks and keys
// come from LDS: nothing is gathered.
__device__ __forceinline__ void fill_tiles_slices(const BinArgs& a, SortSmem& sm, int sb, unsigned pstart, int cnt) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int tx0 = (sb % a.sbx) * 4, ty0 = (sb / a.sbx) * 4;
    const unsigned short* const cov = pay_sorted(sm, cnt);
    const int len = (cnt + 64 * kSortWaves - 1) / (64 * kSortWaves) * 64;
    const int e0 = min(cnt, w * len), e1 = min(cnt, e0 + len);
    // 1. this wave's entries per tile (lane t: tile t)
    unsigned mine = 0u;
    for (int e = e0; e < e1; e += 64 * kFillGroups) {
        unsigned cv[kFillGroups];
#pragma unroll
        for (int q = 0; q < kFillGroups; ++q) cv[q] = e + 64 * q + lane < e1 ? cov[e + 64 * q + lane] : 0u;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            unsigned c = 0u;
#pragma unroll
            for (int q = 0; q < kFillGroups; ++q)
                c += (unsigned)__builtin_popcountll(__builtin_amdgcn_ballot_w64((cv[q] >> t) & 1u));
            if (lane == t) mine += c;
        }
    }
    if (lane < 16) sm.wcnt[w][lane] = mine;
    __syncthreads();
    // 2. tile totals, list starts (row-major tiles of the superblock), ranges
    if (w == 0 && lane < 16) {
        unsigned tot = 0u;
#pragma unroll
        for (int v = 0; v < kSortWaves; ++v) tot += sm.wcnt[v][lane];
        unsigned incl = tot;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const unsigned y = __shfl_up(incl, off, 16);
            if (lane >= off) incl += y;
        }
        const unsigned start = pstart + incl - tot;
        sm.tcnt[lane] = start;
        sm.big[lane] = start + tot;
        const int x = tx0 + (lane & 3), y = ty0 + (lane >> 2);
        if (x < a.cam.tx && y < a.cam.ty) {
            a.ranges[2 * (y * a.cam.tx + x)] = start;
            a.ranges[2 * (y * a.cam.tx + x) + 1] = start + tot;
        }
    }
    __syncthreads();
    // 3. emit the slice; lane t: this wave's next place in tile t, and the tile's end
    unsigned cur = 0u, end = 0u;
    if (lane < 16) {
        cur = sm.tcnt[lane];
        for (int v = 0; v < w; ++v) cur += sm.wcnt[v][lane];
        end = min(sm.big[lane], (unsigned)a.max_pairs);  // P <= max_pairs here; the clamp only guards
    }
    __attribute__((address_space(1))) unsigned* ids = (__attribute__((address_space(1))) unsigned*)a.ids;
    asm volatile("" : "+v"(ids));  // the base in vector registers: the scalar file is full here
    unsigned long long* __restrict__ const keys = a.keys;
    for (int e = e0; e < e1; e += 64 * kFillGroups) {
        unsigned cv[kFillGroups];
        unsigned long long kk[kFillGroups];
#pragma unroll
        for (int q = 0; q < kFillGroups; ++q) {
            const int ee = e + 64 * q + lane;
            cv[q] = ee < e1 ? cov[ee] : 0u;
            kk[q] = sm.xbuf[min(ee, e1 - 1)];
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            unsigned out = (unsigned)__builtin_amdgcn_readlane((int)cur, t);
            const unsigned tend = (unsigned)__builtin_amdgcn_readlane((int)end, t);
            const unsigned long long tk = (unsigned long long)((ty0 + (t >> 2)) * a.cam.tx + tx0 + (t & 3)) << 32;
#pragma unroll
            for (int q = 0; q < kFillGroups; ++q) {
                const bool hit = (cv[q] >> t) & 1u;
                const unsigned long long mask = __builtin_amdgcn_ballot_w64(hit);
                if (hit) {
                    const unsigned pos = out + __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                                         __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
                    if (pos < tend) {  // the counts above use the same test: pos < tend always
                        ids[pos] = (unsigned)(kk[q] & 0xffffffffull);
                        if (keys) keys[pos] = tk | (kk[q] >> 32);
                    }
                }
                out += (unsigned)__builtin_popcountll(mask);
            }
            if (lane == t) cur = out;
        }
    }
}

// The same lists, for small buckets.  Wave t builds the list of tile t
// alone: it counts the bucket's entries whose mask has bit t (one ballot per
// 64 entries), the 16 counts give each tile its start, and a second walk
// over the bucket emits the covering entries in order (one ballot, the
// lane's rank among the covering lanes, one store per 64 entries).  The
// tile, its cursor and its list end stay wave-uniform, and there is one
// workgroup barrier.
static_assert(kSortWaves == 16, "one wave per tile of a 4 x 4-tile superblock");
__device__ __forceinline__ void fill_tiles_per_wave(const BinArgs& a, SortSmem& sm, int sb, unsigned pstart, int cnt) {
    const int lane = threadIdx.x & 63;
    const int t = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int x = (sb % a.sbx) * 4 + (t & 3), y = (sb / a.sbx) * 4 + (t >> 2);
    const unsigned bit = 1u << t;
    const unsigned short* const cov = pay_sorted(sm, cnt);
    // 1. entries of tile t
    unsigned c = 0u;
    for (int e = 0; e < cnt; e += 64 * kFillGroups) {
        unsigned cv[kFillGroups];
#pragma unroll
        for (int q = 0; q < kFillGroups; ++q) cv[q] = e + 64 * q + lane < cnt ? cov[e + 64 * q + lane] : 0u;
#pragma unroll
        for (int q = 0; q < kFillGroups; ++q)
            c += (unsigned)__builtin_popcountll(__builtin_amdgcn_ballot_w64((cv[q] & bit) != 0u));
    }
    if (lane == 0) sm.tcnt[t] = c;
    __syncthreads();
    // 2. the tile's list: after the lists of the superblock's tiles before it (row-major)
    unsigned start = pstart;
#pragma unroll
    for (int v = 0; v < 16; ++v) start += v < t ? sm.tcnt[v] : 0u;
    const unsigned tend = min(start + c, (unsigned)a.max_pairs);  // P <= max_pairs here; the clamp only guards
    if (lane == 0 && x < a.cam.tx && y < a.cam.ty) {
        a.ranges[2 * (y * a.cam.tx + x)] = start;
        a.ranges[2 * (y * a.cam.tx + x) + 1] = start + c;
    }
    // 3. emit the covering entries in bucket order
    const unsigned long long tk = (unsigned long long)(y * a.cam.tx + x) << 32;
    const bool with_keys = a.keys != nullptr;
    // the list bases in vector registers: the scalar file is full here, and
    // scalar copies would be restored from spill lanes before every store
    __attribute__((address_space(1))) unsigned* ids = (__attribute__((address_space(1))) unsigned*)a.ids;
    __attribute__((address_space(1))) unsigned long long* keys =
        (__attribute__((address_space(1))) unsigned long long*)a.keys;
    asm volatile("" : "+v"(ids), "+v"(keys));
    unsigned out = start;
    for (int e = 0; e < cnt; e += 64 * kFillGroups) {
        unsigned cv[kFillGroups];
        unsigned long long kk[kFillGroups];
#pragma unroll
        for (int q = 0; q < kFillGroups; ++q) {
            const int ee = e + 64 * q + lane;
            cv[q] = ee < cnt ? cov[ee] : 0u;
            kk[q] = sm.xbuf[min(ee, cnt - 1)];
        }
#pragma unroll
        for (int q = 0; q < kFillGroups; ++q) {
            const bool hit = (cv[q] & bit) != 0u;
            const unsigned long long mask = __builtin_amdgcn_ballot_w64(hit);
            const unsigned pos = out + __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
            if (hit && pos < tend) {  // the count above uses the same test: pos < tend always
                ids[pos] = (unsigned)(kk[q] & 0xffffffffull);
                if (with_keys) keys[pos] = tk | (kk[q] >> 32);
            }
            out += (unsigned)__builtin_popcountll(mask);
        }
    }
}

// Tile lists from a bucket sorted in LDS with its masks.  Every wave of the
// per-tile form reads the whole bucket, so its time grows with 16 cnt; the
// slice form reads each entry once but pays two barriers and a 16-tile
// bookkeeping per 64 entries, which dominates small buckets.  The small
// buckets are the ones the sort kernel's last workgroups take.
constexpr int kPerWaveFillMax = 2048;
__device__ __forceinline__ void fill_tiles_lds(const BinArgs& a, SortSmem& sm, int sb, unsigned pstart, int cnt) {
    if (cnt <= kPerWaveFillMax)
        fill_tiles_per_wave(a, sm, sb, pstart, cnt);
    else
        fill_tiles_slices(a, sm, sb, pstart, cnt);
}

// Empty tile ranges for every tile of superblock sb: [first, first).
__device__ __forceinline__ void empty_sb_ranges(const BinArgs& a, int sb, unsigned first) {
    const int S = a.S, tx0 = (sb % a.sbx) * S, ty0 = (sb / a.sbx) * S;
    for (int t = threadIdx.x; t < S * S; t += blockDim.x) {
        const int x = tx0 + t % S, y = ty0 + t / S;
        if (x < a.cam.tx && y < a.cam.ty) a.ranges[2 * (y * a.cam.tx + x)] = a.ranges[2 * (y * a.cam.tx + x) + 1] = first;
    }
}

// One workgroup per superblock (largest buckets first): the bucket is sorted
// and the superblock's tile lists and ranges are written from it.  Buckets of
// at most kSortCap keys are sorted in LDS (sort_lds).  Larger buckets are
// first split into 256 bins over the range of their depth bits (a
// most-significant-digit pass through a scratch copy in the free part of the
// pool); runs of consecutive digit bins of at most kSortCap keys are then
// sorted in LDS, in key order, back into the bucket.  Only a bucket with a
// single digit bin beyond kSortCap, or a pool without room for the scratch
// copy, uses the bitonic network in global memory.  If the pairs exceed the
// lists every range is left empty.
__global__ __launch_bounds__(kSortWaves * 64) void k_sb_sort(BinArgs a) {
    __shared__ SortSmem sm;
    if ((int)blockIdx.x >= a.nsb) return;
    const int sb = (int)a.sb_order[blockIdx.x];
    // every per-superblock value at once (one round trip)
    const bool over = a.meta->overflow != 0;
    const int cnt = (int)a.sb_count[sb];
    const unsigned gstart = a.sb_start[sb], pstart = a.sb_pstart[sb];
    if (over) {
        empty_sb_ranges(a, sb, 0u);
        return;
    }
    if (cnt == 0) {
        empty_sb_ranges(a, sb, pstart);
        return;
    }
    unsigned long long* g = a.pool + gstart;
    // units sorted in LDS: the whole bucket, or the chunks of a split bucket
    const unsigned long long* src = g;
    int nunits = 1;
    bool in_lds = true;  // the sorted bucket is also in sm.xbuf
    if (cnt > kSortCap) {
        in_lds = false;
        nunits = split_bucket(a, sm, g, cnt);
        src = a.pool + a.meta->sb_total + gstart;
    }
    // S = 4 buckets of at most kPayCap keys sort their coverage masks along
    const bool lds_fill = in_lds && a.S == 4 && cnt <= kPayCap;
    for (int u = 0; u < nunits; ++u) {
        const int b0 = in_lds ? 0 : (int)sm.chunk_start[u], b1 = in_lds ? cnt : (int)sm.chunk_start[u + 1];
        // a bucket sorted whole stays in LDS for the fill: no copy back
        if (b1 > b0)
            sort_lds(sm, src + b0, in_lds ? nullptr : g + b0, b1 - b0, lds_fill ? a.cov + gstart : nullptr);
    }
    if (lds_fill) {
        fill_tiles_lds(a, sm, sb, pstart, cnt);  // starts after sort_lds's closing LDS barrier
        return;
    }
    if (!in_lds) __threadfence_block();  // the global writes, before the fill reads g
    fill_sb_lists(a, sm, sb, pstart, in_lds ? sm.xbuf : g, cnt);  // starts with a workgroup barrier
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_bin_sort_workspace(const ls2_camera* cam, int32_t n, int64_t max_pairs, size_t* bytes) {
    if (!cam_valid(cam) || n < 0 || max_pairs < 0 || !bytes) return LS2_ERR_ARG;
    if (max_pairs > 0xffffffffll) return LS2_ERR_UNSUPPORTED;  // 32-bit list positions
    *bytes = layout(cam_k(*cam), n, max_pairs).total;
    return LS2_OK;
}

static int bin_sort_impl(const ls2_camera* cam, int32_t n, const float* mean2d, const int32_t* radius,
                         const float* depth, const ProjIO& pj, int64_t max_pairs, uint64_t* keys, uint32_t* ids,
                         uint32_t* tile_ranges, int64_t* num_pairs, void* workspace, size_t workspace_bytes,
                         hipStream_t stream) {
    if (!cam_valid(cam) || n < 0 || max_pairs < 0 || !tile_ranges || !workspace) return LS2_ERR_ARG;
    if (n > 0 && (!mean2d || !radius || !depth)) return LS2_ERR_ARG;
    if (max_pairs > 0 && !ids) return LS2_ERR_ARG;
    if (max_pairs > 0xffffffffll) return LS2_ERR_UNSUPPORTED;
    if (((uintptr_t)workspace & (kAlign - 1)) != 0) return LS2_ERR_ARG;
    const CamK k = cam_k(*cam);
    const Layout lay = layout(k, n, max_pairs);
    if (workspace_bytes < lay.total) return LS2_ERR_ARG;
    const Geo g = geo(k);
    char* ws = static_cast<char*>(workspace);
    BinArgs a;
    a.cam = k;
    a.n = n;
    a.S = g.S;
    a.sbx = g.sbx;
    a.nsb = g.nsb;
    a.max_pairs = max_pairs;
    a.mean2d = mean2d;
    a.radius = radius;
    a.depth = depth;
    a.meta = reinterpret_cast<Meta*>(ws + lay.meta);
    a.sb_count = reinterpret_cast<unsigned*>(ws + lay.sb_count);
    a.sb_pairs = reinterpret_cast<unsigned*>(ws + lay.sb_pairs);
    a.sb_start = reinterpret_cast<unsigned*>(ws + lay.sb_start);
    a.sb_pstart = reinterpret_cast<unsigned*>(ws + lay.sb_pstart);
    a.sb_cursor = reinterpret_cast<unsigned*>(ws + lay.sb_cursor);
    a.sb_order = reinterpret_cast<unsigned*>(ws + lay.sb_order);
    a.rect = reinterpret_cast<ushort4*>(ws + lay.rect);
    a.pool = reinterpret_cast<unsigned long long*>(ws + lay.pool);
    a.cov = reinterpret_cast<unsigned short*>(ws + lay.cov);
    a.ranges = tile_ranges;
    a.ids = ids;
    a.keys = reinterpret_cast<unsigned long long*>(keys);
    a.pj = pj;
    // zero meta, the superblock entry and pair counts and the cursors (contiguous)
    const long long zw = (long long)((lay.sb_start - lay.meta) / sizeof(unsigned));
    const long long zb = (zw + 255) / 256;
    hipLaunchKernelGGL(k_bin_zero, dim3((unsigned)(zb < 1024 ? zb : 1024)), dim3(256), 0, stream,
                       reinterpret_cast<unsigned*>(ws + lay.meta), zw);
    LS2_LAUNCH_CHECK();
    const int per_block = kBinThreads * kBinPerThread;
    const int gblocks = (n + per_block - 1) / per_block;
    if (n > 0) {
        if (pj.means)
            hipLaunchKernelGGL(k_sb_count<true>, dim3(gblocks), dim3(kBinThreads), 0, stream, a);
        else
            hipLaunchKernelGGL(k_sb_count<false>, dim3(gblocks), dim3(kBinThreads), 0, stream, a);
        LS2_LAUNCH_CHECK();
    }
    // the emission also writes the sort kernel's plan: it runs even with no Gaussians
    hipLaunchKernelGGL(k_sb_emit, dim3(gblocks > 0 ? gblocks : 1), dim3(kBinThreads), 0, stream, a);
    LS2_LAUNCH_CHECK();
    // every superblock writes its tiles' ranges (empty ones included)
    hipLaunchKernelGGL(k_sb_sort, dim3(g.nsb), dim3(kSortWaves * 64), 0, stream, a);
    LS2_LAUNCH_CHECK();
    if (num_pairs) {
        Meta h;
        if (hipMemcpyAsync(&h, a.meta, sizeof(Meta), hipMemcpyDeviceToHost, stream) != hipSuccess)
            return LS2_ERR_DEVICE;
        if (hipStreamSynchronize(stream) != hipSuccess) return LS2_ERR_DEVICE;
        *num_pairs = h.P;
        if (h.overflow) return LS2_ERR_CAPACITY;
    }
    return LS2_OK;
}

extern "C" int ls2_bin_sort(const ls2_camera* cam, int32_t n, const float* mean2d, const int32_t* radius,
                            const float* depth, int64_t max_pairs, uint64_t* keys, uint32_t* ids,
                            uint32_t* tile_ranges, int64_t* num_pairs, void* workspace, size_t workspace_bytes,
                            hipStream_t stream) {
    const ProjIO none{};
    return bin_sort_impl(cam, n, mean2d, radius, depth, none, max_pairs, keys, ids, tile_ranges, num_pairs,
                         workspace, workspace_bytes, stream);
}

extern "C" int ls2_project_bin_sort(const ls2_camera* cam, int32_t n, const float* means, const float* scales,
                                    const float* quats, float* mean2d, float* conic, float* depth, int32_t* radius,
                                    int32_t* tiles_touched, int64_t max_pairs, uint64_t* keys, uint32_t* ids,
                                    uint32_t* tile_ranges, int64_t* num_pairs, void* workspace,
                                    size_t workspace_bytes, hipStream_t stream) {
    if (n > 0 && (!means || !scales || !quats || !conic)) return LS2_ERR_ARG;
    ProjIO pj{};
    if (n > 0) pj = ProjIO{means, scales, quats, mean2d, conic, depth, radius, tiles_touched};
    return bin_sort_impl(cam, n, mean2d, radius, depth, pj, max_pairs, keys, ids, tile_ranges, num_pairs,
                         workspace, workspace_bytes, stream);
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
