// ls2_splat_sparse: efficient sparse coefficient splatting (Section 3.4,
// Appendix A Algorithm 1) with the front-to-back rule of Eq. 3.
//
// Mapping on CDNA4:
//   - one wavefront (64 lanes) per (8x8 pixel quadrant of a 16x16 tile,
//     level), one pixel per lane; the waves of a tile walk the same list
//     independently (no workgroup barriers), so each stops as soon as all of
//     its own pixels are saturated (ballot over the lanes).  The level waves
//     of a quadrant recompute the same alphas and transmittance (identical
//     instructions); only level 0's wave writes final_T and last;
//   - the wave stages 64 list entries at a time (one per lane: a gather of
//     the Gaussian's 2D mean, conic, opacity and its K (index, weight) pairs
//     at the wave's level).  The staging lane also tests whether the
//     Gaussian's alpha >= 1/255 ellipse (inflated for rounding) reaches any
//     pixel centre of the quadrant; entries that cannot are dropped by an
//     order-preserving ballot compaction, since every lane would skip them;
//   - every lane then reads each surviving entry back as an LDS broadcast;
//   - only the K stored coefficients are blended, into the pixel's L
//     accumulators held in VGPRs as 32-float vectors addressed with the
//     wave-uniform index through the VGPR index mode.  Staging groups a
//     Gaussian's coefficients by vector (and merges repeated indices), so
//     the blend runs one loop per vector with a wave-uniform trip count: one
//     indexed fused multiply-add per coefficient.  With one level per wave
//     the L accumulators fit in registers at 4 waves per SIMD.
//
// ls2_splat_decode runs the same kernel with Eq. 7's decode as its tail:
// once a wave's 64 pixels are final, their coefficients (rounded to bf16)
// are already spread one pixel per lane, which is what the matrix cores take
// as the B operand of F^T = S^T W^T, after one v_permlane32_swap per register
// (below).  The wave then writes its pixels' D features directly, so the
// coefficient map never travels through HBM, and the feature-map stores of
// finished waves overlap the latency-bound blending of the others.
#include <mutex>

#include "splat_common.h"

namespace ls2 {

typedef float v32f __attribute__((ext_vector_type(32)));
typedef __bf16 bf16x8s __attribute__((ext_vector_type(8)));
typedef unsigned u32x4s __attribute__((ext_vector_type(4)));
typedef float f32x16s __attribute__((ext_vector_type(16)));
typedef float f32x4s __attribute__((ext_vector_type(4)));

typedef float f32x4q __attribute__((ext_vector_type(4)));

// Coefficient output of the splat kernel.  kOutDecodeQuery: the decode tail
// also scores every pixel against the text query (the feature map optional).
enum SplatOut { kOutF32 = 0, kOutBF16 = 1, kOutDecode = 2, kOutDecodeQuery = 3 };

struct SplatArgs {
    CamK cam;
    int n, levels, K, L;
    const unsigned* ranges;
    const unsigned* ids;
    const float* mean2d;
    const float* conic;
    const float* opacity;
    const int* topk_idx;
    const float* topk_w;
    void* coef;  // float32, or bfloat16 (round to nearest even); optional with kOutDecode
    float* final_T;
    int* last;
    // kOutDecode: packed bfloat16 dictionary (k_dict_pack) and the feature map
    int D = 0;
    const unsigned short* dictp = nullptr;
    unsigned short* feat = nullptr;  // optional with kOutDecodeQuery
    // kOutDecodeQuery: texts in bfloat16 [ntext][D] (0 the positive), their
    // float32 norms, the temperature and the relevancy map [levels,H,W]
    const unsigned short* texts = nullptr;
    const float* tnorm = nullptr;
    int ntext = 0;
    float tau = 1.0f;
    float* rel = nullptr;
};

// Feature-map bytes each wave stages at a time in the decode tail: 64 pixels
// x 64 features in bfloat16 (one 128-byte line per pixel).
constexpr int kDecStageBytes = 64 * 64 * 2;

// Staged record (dwords): u, v, A2, B2, C2, o, list position, the first
// code word, then the weights, then the remaining code words.
//
// The K coefficients go to accumulator vector h = index / 32 (NV vectors of
// 32).  Vectors 2p and 2p + 1 share slot array p (KMAX weight slots): vector
// 2p fills it from the front, vector 2p + 1 from the back, each in slot
// order, so every slot a blend reads sits at a compile-time position.  Code
// word 0 of array p holds slots 0-3 as 5-bit indices within the vector (bits
// 0-19), the front count (bits 24-27) and the back count (bits 28-31); code
// word 1 (KMAX = 8) holds slots 4-7.  Repeated indices of a Gaussian are
// merged into their first slot (the sum of their weights, in slot order).
// A2 = -0.5 A log2(e), B2 = -B log2(e), C2 = -0.5 C log2(e): the Gaussian's
// exponent in base 2 is A2 dx^2 + B2 dx dy + C2 dy^2.
template <int KMAX, int NV>
struct Rec {
    static_assert(KMAX == 4 || KMAX == 8, "weights are read as float4");
    static constexpr int NP = (NV + 1) / 2;  // slot arrays
    static constexpr int CW = KMAX / 4;      // code words per slot array
    static constexpr int POS = 6;
    static constexpr int CODE0 = 7;          // code word 0 of slot array 0
    static constexpr int W = 8;              // weights of slot array p at W + KMAX p
    static constexpr int CODE = W + NP * KMAX;  // code word q of array p (but array 0, word 0) at CODE + p CW + q - 1
    static constexpr int RAW = CODE + NP * CW - 1;
    static constexpr int STRIDE = (RAW + 3) & ~3;  // 16-byte aligned records
    __device__ static int code_at(int p, int q) { return p == 0 && q == 0 ? CODE0 : CODE + p * CW + q - 1; }
};

// Decode tail of one wave: F = W S (Eq. 7) for the wave's 64 pixels (lane p
// holds pixel p's L accumulators), written as bfloat16 rows of D features.
//
// MFMA 32x32x16 bf16 computes the transposed tile F^T[32 features x 32
// pixels] with A = S^T (lane (c, h): feature c, k = 16 ks + 8 h + [0,8)) and
// B = W^T (lane (c, h): pixel c of the 32-pixel tile, the same k).  Lane p
// owns pixel p; with X = its k-range 16 ks + [0,8) and Y = 16 ks + [8,16),
// v_permlane32_swap(X, Y) leaves exactly the B operand of pixel tile 0
// (lanes 0-31 keep X, lanes 32-63 receive Y of lane p - 32) in X and that of
// pixel tile 1 (lanes 0-31 receive X of lane p + 32, lanes 32-63 keep Y) in
// Y.  The k-steps accumulate in the same order and with the same operands as
// ls2_dict_decode's bf16 kernel, so the features are bit-identical to
// splatting a bfloat16 map and decoding it.  Every lane must be active;
// lanes outside the image hold zero coefficients and store nothing.
//
// dsrc: the packed dictionary (k_dict_pack), in HBM or in LDS.  The wave
// stages CF features of its 64 pixels at a time in st (64 CF 2 bytes) and
// writes them as CF-feature runs of each pixel.
//
// QRY: while each chunk is staged, the four 16-pixel blocks of the wave are
// scored exactly as ls2_query scores a bf16 feature map: MFMA 16x16x32 bf16
// with A = the block's features (lane (r, g): pixel r, features 32 ks + 8 g
// + [0,8)) and B = the bf16 texts, plus the Gram tile of A for the squared
// norms, accumulated over the k-steps in increasing order.  Every output
// element of these products depends only on its own row and column, so the
// relevancy equals ls2_query on the written map bit for bit.
template <int NV, int CF, bool QRY>
__device__ __forceinline__ void decode_tail(const SplatArgs& a, const v32f (&acc)[NV], char* st, int lane, int lv0,
                                            int qx0, int qy0, const unsigned short* dsrc) {
    constexpr int KS = 2 * NV;   // k-steps of 16
    constexpr int U = CF / 8;    // 16-byte units per pixel and chunk
    constexpr int FT = CF / 32;  // feature tiles per chunk
    constexpr int PPI = 64 / U;  // pixels per store instruction
    static_assert(CF == 32 || CF == 64, "decode_tail: 32- or 64-feature chunks");
    const int col = lane & 31, half = lane >> 5;
    // A operand of lane l at k-step ks of feature tile ft: 16-byte unit
    // (ft KS + ks) 64 + l of the packed dictionary (through L2).  Both tiles
    // of a chunk are loaded at once: the first chunk's before the operand
    // conversion, each later chunk's as soon as the previous chunk's results
    // are staged, so the L2 latency hides behind the store phase.  With QRY,
    // whose scoring needs those registers, each tile loads just before use.
    const u32x4s* dv = reinterpret_cast<const u32x4s*>(dsrc) + lane;
    auto load_tile = [&](int ft, u32x4s (&o)[KS]) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) o[ks] = dv[(ft * KS + ks) * 64];
    };
    u32x4s sa[FT][KS];  // QRY: one tile at a time, in sa[0]
#pragma unroll
    for (int cc = 0; cc < (QRY ? 1 : FT); ++cc) load_tile(cc, sa[cc]);
    bf16x8s wb[2][KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int h = ks >> 1, jb = (ks & 1) * 16;
        u32x4s x, y;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const unsigned lo = bf16_pair(acc[h][jb + 2 * q], acc[h][jb + 2 * q + 1]);
            const unsigned hi = bf16_pair(acc[h][jb + 8 + 2 * q], acc[h][jb + 9 + 2 * q]);
            const auto r = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
            x[q] = r[0];
            y[q] = r[1];
        }
        wb[0][ks] = __builtin_bit_cast(bf16x8s, x);
        wb[1][ks] = __builtin_bit_cast(bf16x8s, y);
    }
    const int D = a.D, nft = D / 32;
    const int W = a.cam.W, H = a.cam.H;
    // store phase: instruction i covers pixels PPI i + pi (quadrant rows
    // (8 / U) i + yo, column xo), lane writing 16-byte unit su of its pixel
    const int pi = lane / U, su = lane % U;
    const int xo = pi & 7, yo = pi >> 3;
    const bool xin = qx0 + xo < W;
    const size_t rstride = (size_t)W * D;
    unsigned short* fbase = a.feat + ((size_t)lv0 * H + qy0 + yo) * rstride + (size_t)(qx0 + xo) * D + su * 8;
    const bool store = !QRY || a.feat != nullptr;
    // QRY: lane (r16, g) of the 16x16x32 products; dot and Gram tiles of the
    // four 16-pixel blocks
    const int r16 = lane & 15, g16 = lane >> 4;
    const bool tcol = QRY && r16 < a.ntext;
    f32x4q dq[QRY ? 4 : 1], gq[QRY ? 4 : 1];
#pragma unroll
    for (int rb = 0; rb < (QRY ? 4 : 1); ++rb) dq[rb] = gq[rb] = (f32x4q){0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < D / CF; ++c) {
#pragma unroll
        for (int cc = 0; cc < FT; ++cc) {
            if (QRY && FT * c + cc > 0) load_tile(FT * c + cc, sa[0]);
            f32x16s f0 = {}, f1 = {};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const bf16x8s av = __builtin_bit_cast(bf16x8s, sa[QRY ? 0 : cc][ks]);
                f0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, wb[0][ks], f0, 0, 0, 0);
                f1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, wb[1][ks], f1, 0, 0, 0);
            }
            // lane (c, h) holds pixel 32 t + c, features 32 ft + 8 g + 4 h + [0,4):
            // 16-byte unit 4 cc + g of the pixel's chunk, stored at unit
            // (4 cc + g) ^ (pixel % U) to spread the LDS banks
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int u = ((4 * cc + g) ^ (col & (U - 1))) * 16 + half * 8;
                *reinterpret_cast<uint2*>(st + col * (U * 16) + u) =
                    make_uint2(bf16_pair(f0[4 * g], f0[4 * g + 1]), bf16_pair(f0[4 * g + 2], f0[4 * g + 3]));
                *reinterpret_cast<uint2*>(st + (32 + col) * (U * 16) + u) =
                    make_uint2(bf16_pair(f1[4 * g], f1[4 * g + 1]), bf16_pair(f1[4 * g + 2], f1[4 * g + 3]));
            }

        }
        // the chunk's operands are consumed: the next chunk's load from L2
        // while this chunk is scored and stored
        if (!QRY && c + 1 < D / CF)
#pragma unroll
            for (int cc = 0; cc < FT; ++cc) load_tile(FT * (c + 1) + cc, sa[cc]);
        wave_lds_order();
        if (QRY) {
            const bf16x8s zero8 = {};
#pragma unroll
            for (int kk = 0; kk < CF / 32; ++kk) {
                const bf16x8s tb = tcol ? *reinterpret_cast<const bf16x8s*>(a.texts + (size_t)r16 * D + c * CF +
                                                                             kk * 32 + g16 * 8)
                                        : zero8;
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const int p = 16 * rb + r16;
                    const bf16x8s fa = *reinterpret_cast<const bf16x8s*>(
                        st + p * (U * 16) + (((4 * kk + g16) ^ (p & (U - 1))) * 16));
                    dq[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, tb, dq[rb], 0, 0, 0);
                    gq[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fa, gq[rb], 0, 0, 0);
                }
            }
        }
        if (store) {
            // every staged line read first (one LDS wait), then the stores
            f32x4s v[U];
#pragma unroll
            for (int i = 0; i < U; ++i) {
                const int p = PPI * i + pi;  // p % U == pi % U
                v[i] = *reinterpret_cast<const f32x4s*>(st + p * (U * 16) + ((su ^ (pi & (U - 1))) * 16));
            }
#pragma unroll
            for (int i = 0; i < U; ++i)
                if (xin && qy0 + (8 / U) * i + yo < H)
                    __builtin_nontemporal_store(
                        v[i], reinterpret_cast<f32x4s*>(fbase + (size_t)((8 / U) * i) * rstride + c * CF));
        }
        wave_lds_order();  // the next chunk overwrites the staged lines
    }
    if (QRY) {
        // per block: the dot tile (lane: text r16, pixels 4 g + i) and the
        // Gram diagonal to LDS, then lanes 0..15 score their pixel
        float* dots_w = reinterpret_cast<float*>(st);  // [16 pixels][17]
        float* nrm_w = dots_w + 16 * 17;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const int i = r16 - g16 * 4;
            if (i >= 0 && i < 4) nrm_w[r16] = gq[rb][i];
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) dots_w[(g16 * 4 + ii) * 17 + r16] = dq[rb][ii];
            wave_lds_order();
            if (lane < 16) {
                const int p = 16 * rb + lane;
                const int x = qx0 + (p & 7), y = qy0 + (p >> 3);
                if (x < W && y < H)
                    a.rel[((size_t)lv0 * H + y) * W + x] =
                        lerf_relevancy(dots_w + lane * 17, nrm_w[lane], a.tnorm, a.ntext, a.tau);
            }
            wave_lds_order();
        }
    }
}

// EXACT: K == KMAX is known at compile time.  NV = L / 32 accumulator vectors.
// OUT: kOutF32 / kOutBF16 write the coefficient map; kOutDecode writes the
// feature map (and the bfloat16 coefficient map if a.coef is set).
// One work item: the wave's (quadrant `slot & 3`, level `slot >> 2`) of
// `tile`, one pixel per lane.  stage: the wave's LDS (records, and the decode
// tail's staging of CF-feature chunks); dsrc: the packed dictionary.
template <int NV, int KMAX, bool EXACT, int OUT, int CF>
__device__ __forceinline__ void splat_item(const SplatArgs& a, int tile, int slot, int lane, float* stage,
                                           const unsigned short* dsrc) {
    using R = Rec<KMAX, NV>;
    const CamK& cam = a.cam;
    const int quad = slot & 3, lv0 = slot >> 2;
    const int tx = tile % cam.tx, ty = tile / cam.tx;
    const int qx0 = tx * kTile + (quad & 1) * 8, qy0 = ty * kTile + (quad >> 1) * 8;
    if (qx0 >= cam.W || qy0 >= cam.H) return;  // quadrant fully outside the image
    const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
    const bool inside = px < cam.W && py < cam.H;
    const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
    // pixel-centre box of the quadrant's pixels inside the image
    const float bx0 = (float)qx0 + 0.5f, by0 = (float)qy0 + 0.5f;
    const float bx1 = (float)min(qx0 + 7, cam.W - 1) + 0.5f, by1 = (float)min(qy0 + 7, cam.H - 1) + 0.5f;

    const unsigned start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const int K = EXACT ? KMAX : a.K, L = a.L;
    const int lstride = a.levels;  // levels per Gaussian in topk_idx / topk_w
    const int lmask = L - 1;
    const unsigned long long lt = (1ull << lane) - 1ull;

    v32f acc[NV];
#pragma unroll
    for (int h = 0; h < NV; ++h) acc[h] = (v32f){};

    float T = 1.0f;
    int last = 0;
    bool active = inside;

    // Software pipeline over 64-entry batches: while batch b is processed,
    // the records of batch b + 64 and the ids of batch b + 128 are in flight.
    constexpr int PK = KMAX;  // the (index, weight) pairs are prefetched too
    const unsigned kBad = 0xffffffffu;
    auto fetch_id = [&](unsigned pos) -> unsigned { return pos < end ? a.ids[pos] : kBad; };
    unsigned nid = fetch_id(start + lane);           // ids of the batch staged next
    unsigned nid2 = fetch_id(start + 64 + lane);     // ids of the batch after
    float n_mu = 0.f, n_mv = 0.f, n_cA = 0.f, n_cB = 0.f, n_cC = 0.f, n_op = 0.f;
    int n_ix[PK];
    float n_w[PK];
    auto fetch_rec = [&](unsigned id) {
        if (id < (unsigned)a.n) {  // an id outside [0, n) can only come from a corrupted list
            const float2 m = reinterpret_cast<const float2*>(a.mean2d)[id];
            n_mu = m.x;
            n_mv = m.y;
            n_cA = a.conic[3 * id];
            n_cB = a.conic[3 * id + 1];
            n_cC = a.conic[3 * id + 2];
            n_op = a.opacity[id];
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const size_t o = ((size_t)id * lstride + lv0) * K + k;
                n_ix[k] = k < K ? a.topk_idx[o] : 0;
                n_w[k] = k < K ? a.topk_w[o] : 0.0f;
            }
        } else {
            n_op = 0.0f;
        }
    };
    fetch_rec(nid);

    for (unsigned b = start; b < end; b += 64) {
        if (__builtin_amdgcn_ballot_w64(active) == 0) break;
        const int nb = (int)min(64u, end - b);
        // ---- stage: lane j holds entry b + j (fetched one batch ago)
        const unsigned id = nid;
        const float mu = n_mu, mv = n_mv, cA = n_cA, cB = n_cB, cC = n_cC, op = n_op;
        int c_ix[PK];
        float c_w[PK];
#pragma unroll
        for (int q = 0; q < PK; ++q) {
            c_ix[q] = n_ix[q];
            c_w[q] = n_w[q];
        }
        const bool keep = lane < nb && id < (unsigned)a.n && may_touch(mu, mv, cA, cB, cC, op, bx0, bx1, by0, by1);
        // prefetch: records of batch b + 64, ids of batch b + 128
        nid = nid2;
        fetch_rec(nid);
        nid2 = fetch_id(b + 128 + lane);
        const unsigned long long kmask = __builtin_amdgcn_ballot_w64(keep);
        const int nkeep = __builtin_popcountll(kmask);
        wave_lds_order();  // single-wave workgroup: the previous batch's stage reads are done
        if (keep) {
            float* r = stage + __builtin_popcountll(kmask & lt) * R::STRIDE;
            r[0] = mu;
            r[1] = mv;
            r[2] = -0.5f * kLog2e * cA;
            r[3] = -kLog2e * cB;
            r[4] = -0.5f * kLog2e * cC;
            r[5] = op;
            reinterpret_cast<unsigned*>(r)[R::POS] = b - start + lane;
            unsigned ix[KMAX];
            float wv[KMAX];
            bool live[KMAX];
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                live[k] = k < K;
                ix[k] = k < K ? (unsigned)(c_ix[k] & lmask) : 0u;
                wv[k] = k < K ? c_w[k] : 0.0f;
            }
            // merge repeated indices into their first slot (the sum of their
            // weights, in slot order)
#pragma unroll
            for (int k = 1; k < KMAX; ++k)
#pragma unroll
                for (int k2 = 0; k2 < k; ++k2)
                    if (live[k2] && live[k] && ix[k2] == ix[k]) {
                        wv[k2] += wv[k];
                        live[k] = false;
                    }
            // slot arrays: vector 2p from the front, vector 2p + 1 from the back
            unsigned code[R::NP][R::CW];
            int nf[R::NP], nb[R::NP];
#pragma unroll
            for (int p = 0; p < R::NP; ++p) {
                nf[p] = nb[p] = 0;
#pragma unroll
                for (int q = 0; q < R::CW; ++q) code[p][q] = 0u;
#pragma unroll
                for (int q = 0; q < KMAX; ++q) r[R::W + p * KMAX + q] = 0.0f;
            }
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                if (!live[k]) continue;
                const int h = (int)(ix[k] >> 5);
#pragma unroll
                for (int p = 0; p < R::NP; ++p) {
                    if ((h >> 1) != p) continue;
                    const int sl = (h & 1) ? KMAX - 1 - nb[p]++ : nf[p]++;
                    r[R::W + p * KMAX + sl] = wv[k];
#pragma unroll
                    for (int q = 0; q < R::CW; ++q)
                        if ((sl >> 2) == q) code[p][q] |= (ix[k] & 31u) << (5 * (sl & 3));
                }
            }
            unsigned* ru = reinterpret_cast<unsigned*>(r);
#pragma unroll
            for (int p = 0; p < R::NP; ++p) {
                code[p][0] |= (unsigned)nf[p] << 24 | (unsigned)nb[p] << 28;
#pragma unroll
                for (int q = 0; q < R::CW; ++q) ru[R::code_at(p, q)] = code[p][q];
            }
        }
        wave_lds_order();  // single-wave workgroup: orders the LDS writes before the reads

        // Evaluate UNR staged entries at a time: their alphas are independent,
        // so the LDS reads and exponentials of the group overlap; the
        // transmittance logic and the blends then run in list order.
        constexpr int UNR = 4;
        for (int j = 0; j < nkeep; j += UNR) {
            float4 h0[UNR], h1[UNR];
            float p2[UNR], g[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const float* r = stage + min(j + u, 63) * R::STRIDE;  // past nkeep: read, never used
                h0[u] = *reinterpret_cast<const float4*>(r);
                h1[u] = *reinterpret_cast<const float4*>(r + 4);
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const float dx = h0[u].x - pxc, dy = h0[u].y - pyc;
                p2[u] = gauss_power2(h0[u].z, h0[u].w, h1[u].x, dx, dy);
                g[u] = h1[u].y * fast_exp2(p2[u]);
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                if (j + u >= nkeep) break;  // wave-uniform
                const float* r = stage + (j + u) * R::STRIDE;
                const float alpha = fminf(0.99f, g[u]);
                const float c = alpha * T;       // blend weight e_i = alpha_i T_i (Eq. 7)
                const float testT = T - c;       // T (1 - alpha)
                const bool hit = active && p2[u] <= 0.0f && alpha >= (1.0f / 255.0f);
                const bool stop = hit && testT < 1e-4f;
                const bool contrib = hit && !stop;
                active = active && !stop;
                if (contrib) {  // divergent: only contributing lanes blend (exec mask)
#pragma unroll
                    for (int p = 0; p < R::NP; ++p) {
                        unsigned cw[R::CW];
#pragma unroll
                        for (int q = 0; q < R::CW; ++q)
                            cw[q] = __builtin_amdgcn_readfirstlane(
                                p == 0 && q == 0 ? __float_as_uint(h1[u].w)
                                                 : reinterpret_cast<const unsigned*>(r)[R::code_at(p, q)]);
                        f32x4s wq[KMAX / 4];
#pragma unroll
                        for (int q = 0; q < KMAX / 4; ++q)
                            wq[q] = *reinterpret_cast<const f32x4s*>(r + R::W + p * KMAX + 4 * q);
                        const int nfr = (int)(cw[0] >> 24) & 15, nbk = (int)(cw[0] >> 28);
                        // vector 2p: slots 0, 1, ... (front)
#pragma unroll
                        for (int q = 0; q < KMAX; ++q) {
                            if (q >= nfr) break;  // wave-uniform
                            const unsigned jl = (cw[q >> 2] >> (5 * (q & 3))) & 31u;
                            acc[2 * p][jl] = fmaf(wq[q >> 2][q & 3], c, acc[2 * p][jl]);
                        }
                        if (2 * p + 1 < NV) {
                            // vector 2p + 1: slots KMAX - 1, KMAX - 2, ... (back)
#pragma unroll
                            for (int q = 0; q < KMAX; ++q) {
                                if (q >= nbk) break;  // wave-uniform
                                const int sl = KMAX - 1 - q;
                                const unsigned jl = (cw[sl >> 2] >> (5 * (sl & 3))) & 31u;
                                acc[(2 * p + 1) % NV][jl] = fmaf(wq[sl >> 2][sl & 3], c, acc[(2 * p + 1) % NV][jl]);
                            }
                        }
                    }
                    T = testT;
                    last = __float_as_int(h1[u].z) + 1;  // record dword POS: list position
                }
            }
            if (__builtin_amdgcn_ballot_w64(active) == 0) break;
        }
    }

    // the pixel's outputs first: the decode tail below then holds no
    // accumulator beyond its bfloat16 operands
    if (inside) {
        const size_t HW = (size_t)cam.W * cam.H;
        const size_t pix = (size_t)py * cam.W + px;
        const size_t row = ((size_t)lv0 * HW + pix) * (size_t)(NV * 32);
        if (OUT >= kOutDecode && !a.coef) {
            // feature map only
        } else if (OUT != kOutF32) {
            uint4* dst = reinterpret_cast<uint4*>(static_cast<unsigned short*>(a.coef) + row);
#pragma unroll
            for (int h = 0; h < NV; ++h)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    dst[h * 4 + q] = make_uint4(
                        bf16_pair(acc[h][8 * q], acc[h][8 * q + 1]), bf16_pair(acc[h][8 * q + 2], acc[h][8 * q + 3]),
                        bf16_pair(acc[h][8 * q + 4], acc[h][8 * q + 5]),
                        bf16_pair(acc[h][8 * q + 6], acc[h][8 * q + 7]));
        } else {
            float4* dst = reinterpret_cast<float4*>(static_cast<float*>(a.coef) + row);
#pragma unroll
            for (int h = 0; h < NV; ++h)
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    dst[h * 8 + q] =
                        make_float4(acc[h][4 * q], acc[h][4 * q + 1], acc[h][4 * q + 2], acc[h][4 * q + 3]);
        }
        if (lv0 == 0) {  // every level wave of the quadrant computes the same T and last
            if (a.final_T) a.final_T[pix] = T;
            if (a.last) a.last[pix] = last;
        }
    }
    if (OUT == kOutDecode || OUT == kOutDecodeQuery) {
        wave_lds_order();  // the record reads of the last batch are done
        decode_tail<NV, CF, OUT == kOutDecodeQuery>(a, acc, reinterpret_cast<char*>(stage), lane, lv0, qx0, qy0, dsrc);
    }
}

// One wave per workgroup and work item (the hardware dispatcher balances the
// items).  The decode form reads the packed dictionary through L2: keeping it
// in LDS would need workgroups of many waves sharing one copy, which leaves
// no room for 128-byte output staging (32-feature staging alone costs more
// than the L2 reads save).
template <int NV, int KMAX, bool EXACT, int OUT>
__global__ __launch_bounds__(64, NV <= 2 ? 4 : 2) void k_splat_sparse(SplatArgs a) {
    using R = Rec<KMAX, NV>;
    constexpr int REC4 = 64 * R::STRIDE / 4;
    constexpr int STAGE4 = OUT >= kOutDecode && kDecStageBytes / 16 > REC4 ? kDecStageBytes / 16 : REC4;
    __shared__ float4 stage4[STAGE4];
    int tile, slot;
    xcd_remap(blockIdx.x, gridDim.x, 4 * a.levels, tile, slot);
    if (tile >= a.cam.tx * a.cam.ty) return;
    splat_item<NV, KMAX, EXACT, OUT, 64>(a, tile, slot, threadIdx.x, reinterpret_cast<float*>(stage4), a.dictp);
}

template <int NV, int KMAX, bool EXACT>
static void launch_splat_out(const SplatArgs& a, int out, dim3 grid, hipStream_t stream) {
    if (out == kOutDecodeQuery)
        hipLaunchKernelGGL((k_splat_sparse<NV, KMAX, EXACT, kOutDecodeQuery>), grid, dim3(64), 0, stream, a);
    else if (out == kOutDecode)
        hipLaunchKernelGGL((k_splat_sparse<NV, KMAX, EXACT, kOutDecode>), grid, dim3(64), 0, stream, a);
    else if (out == kOutBF16)
        hipLaunchKernelGGL((k_splat_sparse<NV, KMAX, EXACT, kOutBF16>), grid, dim3(64), 0, stream, a);
    else
        hipLaunchKernelGGL((k_splat_sparse<NV, KMAX, EXACT, kOutF32>), grid, dim3(64), 0, stream, a);
}

template <int NV, int KMAX>
static int launch_splat(const SplatArgs& a, int out, hipStream_t stream) {
    const int ntiles = a.cam.tx * a.cam.ty;
    const dim3 grid((unsigned)round_up8(ntiles * 4 * a.levels));
    if (a.K == KMAX)
        launch_splat_out<NV, KMAX, true>(a, out, grid, stream);
    else
        launch_splat_out<NV, KMAX, false>(a, out, grid, stream);
    LS2_LAUNCH_CHECK();
    return LS2_OK;
}

template <int NV>
static int launch_splat_k(const SplatArgs& a, int out, hipStream_t stream) {
    return a.K > 4 ? launch_splat<NV, 8>(a, out, stream) : launch_splat<NV, 4>(a, out, stream);
}

static int launch_splat_l(const SplatArgs& a, int out, hipStream_t stream) {
    if (a.L == 32) return launch_splat_k<1>(a, out, stream);
    if (a.L == 64) return launch_splat_k<2>(a, out, stream);
    return launch_splat_k<4>(a, out, stream);
}

// Dictionary [L,D] float32 -> the decode tail's A operands in bfloat16
// (nearest even): 16-byte unit ((ft KS + ks) 2 + h) 32 + c holds
// S[16 ks + 8 h + e][32 ft + c], e = 0..7, so the 64 lanes of one k-step read
// 1 KB contiguously.
__global__ __launch_bounds__(256) void k_dict_pack(int L, int D, const float* __restrict__ dict,
                                                   unsigned short* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L * D) return;
    const int KS = L / 16;
    const int e = i & 7, unit = i >> 3;
    const int c = unit & 31, h = (unit >> 5) & 1, r = unit >> 6;
    const int ks = r % KS, ft = r / KS;
    out[i] = __builtin_bit_cast(unsigned short, (__bf16)dict[(size_t)(16 * ks + 8 * h + e) * D + 32 * ft + c]);
}

}  // namespace ls2

using namespace ls2;

extern "C" int ls2_splat_sparse(const ls2_camera* cam, int32_t n, int32_t levels, int32_t K, int32_t L,
                                const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                                const float* conic, const float* opacity, const int32_t* topk_idx,
                                const float* topk_w, void* coef, int32_t coef_dtype, float* final_T,
                                int32_t* last, hipStream_t stream) {
    if (!cam_valid(cam) || n < 0 || levels < 1 || K < 1 || L < 1 || K > L) return LS2_ERR_ARG;
    if (!tile_ranges || !coef) return LS2_ERR_ARG;
    if (coef_dtype != LS2_F32 && coef_dtype != LS2_BF16) return LS2_ERR_ARG;
    if (!aligned16(coef)) return LS2_ERR_ARG;
    if (n > 0 && (!ids || !mean2d || !conic || !opacity || !topk_idx || !topk_w)) return LS2_ERR_ARG;
    if (!(L == 32 || L == 64 || L == 128) || K > 8 || levels > 3 || levels * L > 192) return LS2_ERR_UNSUPPORTED;
    if (const int st = check_code_indices((long long)n * levels * K, L, topk_idx, stream)) return st;
    SplatArgs a;
    a.cam = cam_k(*cam);
    a.n = n;
    a.levels = levels;
    a.K = K;
    a.L = L;
    a.ranges = tile_ranges;
    a.ids = ids;
    a.mean2d = mean2d;
    a.conic = conic;
    a.opacity = opacity;
    a.topk_idx = topk_idx;
    a.topk_w = topk_w;
    a.coef = coef;
    a.final_T = final_T;
    a.last = last;
    return launch_splat_l(a, coef_dtype == LS2_BF16 ? kOutBF16 : kOutF32, stream);
}

// Texts of the query: bfloat16 copies [ntext][D] and float32 norms, the
// norms summed in the same order as ls2_query's (lane-strided, then an xor
// butterfly), so that the relevancy matches it bit for bit.
__global__ __launch_bounds__(256) void k_text_pack(int D, int ntext, const float* __restrict__ pos,
                                                   const float* __restrict__ neg, unsigned short* __restrict__ texts,
                                                   float* __restrict__ tnorm) {
    for (int i = threadIdx.x; i < ntext * D; i += blockDim.x) {
        const int j = i / D, d = i - j * D;
        const float v = j == 0 ? pos[d] : neg[(size_t)(j - 1) * D + d];
        texts[i] = __builtin_bit_cast(unsigned short, (__bf16)v);
    }
    if (threadIdx.x < 64) {
        for (int j = 0; j < ntext; ++j) {
            float s = 0.f;
            const float* t = j == 0 ? pos : neg + (size_t)(j - 1) * D;
            for (int d = threadIdx.x; d < D; d += 64) s += t[d] * t[d];
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            if (threadIdx.x == 0) tnorm[j] = fmaxf(sqrtf(s), 1e-12f);
        }
    }
}

static size_t al256s(size_t x) { return (x + 255) & ~(size_t)255; }

// Validation and set-up shared by the one-pass entry points; launches the
// dictionary repack.
static int splat_decode_setup(SplatArgs& a, const ls2_camera* cam, int32_t n, int32_t levels, int32_t K, int32_t L,
                              int32_t D, const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                              const float* conic, const float* opacity, const int32_t* topk_idx, const float* topk_w,
                              const float* dict, void* feat, bool feat_required, void* coef, float* final_T,
                              int32_t* last, void* workspace, size_t workspace_bytes, size_t ws_need,
                              hipStream_t stream) {
    if (!cam_valid(cam) || n < 0 || levels < 1 || K < 1 || L < 1 || K > L || D < 1) return LS2_ERR_ARG;
    if (!tile_ranges || (feat_required && !feat) || !dict || !workspace) return LS2_ERR_ARG;
    if (!aligned16(feat) || !aligned16(coef) || !aligned16(workspace)) return LS2_ERR_ARG;
    if (n > 0 && (!ids || !mean2d || !conic || !opacity || !topk_idx || !topk_w)) return LS2_ERR_ARG;
    if (!(L == 32 || L == 64 || L == 128) || K > 8 || levels > 3 || levels * L > 192) return LS2_ERR_UNSUPPORTED;
    if (D % 64 != 0 || D > 1024) return LS2_ERR_UNSUPPORTED;
    if (workspace_bytes < ws_need) return LS2_ERR_ARG;
    if (const int st = check_code_indices((long long)n * levels * K, L, topk_idx, stream)) return st;
    unsigned short* dictp = static_cast<unsigned short*>(workspace);
    hipLaunchKernelGGL(k_dict_pack, dim3((unsigned)((L * D + 255) / 256)), dim3(256), 0, stream, L, D, dict, dictp);
    LS2_LAUNCH_CHECK();
    a.cam = cam_k(*cam);
    a.n = n;
    a.levels = levels;
    a.K = K;
    a.L = L;
    a.ranges = tile_ranges;
    a.ids = ids;
    a.mean2d = mean2d;
    a.conic = conic;
    a.opacity = opacity;
    a.topk_idx = topk_idx;
    a.topk_w = topk_w;
    a.coef = coef;
    a.final_T = final_T;
    a.last = last;
    a.D = D;
    a.dictp = dictp;
    a.feat = static_cast<unsigned short*>(feat);
    return LS2_OK;
}

extern "C" int ls2_splat_decode_workspace(int32_t L, int32_t D, size_t* bytes) {
    if (!bytes || L < 1 || D < 1) return LS2_ERR_ARG;
    if (!(L == 32 || L == 64 || L == 128) || D % 64 != 0 || D > 1024) return LS2_ERR_UNSUPPORTED;
    *bytes = (size_t)L * D * 2;  // the packed dictionary
    return LS2_OK;
}

extern "C" int ls2_splat_decode(const ls2_camera* cam, int32_t n, int32_t levels, int32_t K, int32_t L, int32_t D,
                                const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                                const float* conic, const float* opacity, const int32_t* topk_idx,
                                const float* topk_w, const float* dict, void* feat, void* coef, float* final_T,
                                int32_t* last, void* workspace, size_t workspace_bytes, hipStream_t stream) {
    SplatArgs a;
    const int st = splat_decode_setup(a, cam, n, levels, K, L, D, tile_ranges, ids, mean2d, conic, opacity, topk_idx,
                                      topk_w, dict, feat, true, coef, final_T, last, workspace, workspace_bytes,
                                      (size_t)(L > 0 ? L : 0) * (D > 0 ? D : 0) * 2, stream);
    if (st != LS2_OK) return st;
    return launch_splat_l(a, kOutDecode, stream);
}

extern "C" int ls2_splat_decode_query_workspace(int32_t L, int32_t D, int32_t n_neg, size_t* bytes) {
    if (!bytes || L < 1 || D < 1 || n_neg < 1) return LS2_ERR_ARG;
    if (!(L == 32 || L == 64 || L == 128) || D % 64 != 0 || D > 1024 || n_neg > 8) return LS2_ERR_UNSUPPORTED;
    // packed dictionary, bf16 texts, text norms
    *bytes = al256s((size_t)L * D * 2) + al256s((size_t)(1 + n_neg) * D * 2) + 64;
    return LS2_OK;
}

// The query frame given its scratch: the packed dictionary at w, the bf16
// texts and their norms after it (the layout ls2_splat_decode_query_workspace
// sizes).
static int splat_decode_query_run(const ls2_camera* cam, int32_t n, int32_t levels, int32_t K, int32_t L, int32_t D,
                                  const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                                  const float* conic, const float* opacity, const int32_t* topk_idx,
                                  const float* topk_w, const float* dict, const float* pos, int32_t n_neg,
                                  const float* neg, float tau, float* relevancy, void* feat, void* coef,
                                  float* final_T, int32_t* last, void* workspace, size_t workspace_bytes,
                                  size_t need, hipStream_t stream) {
    SplatArgs a;
    int st = splat_decode_setup(a, cam, n, levels, K, L, D, tile_ranges, ids, mean2d, conic, opacity, topk_idx,
                                topk_w, dict, feat, false, coef, final_T, last, workspace, workspace_bytes, need,
                                stream);
    if (st != LS2_OK) return st;
    char* w = static_cast<char*>(workspace) + al256s((size_t)L * D * 2);
    unsigned short* texts = reinterpret_cast<unsigned short*>(w);
    float* tnorm = reinterpret_cast<float*>(w + al256s((size_t)(1 + n_neg) * D * 2));
    hipLaunchKernelGGL(k_text_pack, dim3(1), dim3(256), 0, stream, D, 1 + n_neg, pos, neg, texts, tnorm);
    LS2_LAUNCH_CHECK();
    a.texts = texts;
    a.tnorm = tnorm;
    a.ntext = 1 + n_neg;
    a.tau = tau;
    a.rel = relevancy;
    return launch_splat_l(a, kOutDecodeQuery, stream);
}

extern "C" int ls2_splat_decode_query(const ls2_camera* cam, int32_t n, int32_t levels, int32_t K, int32_t L,
                                      int32_t D, const uint32_t* tile_ranges, const uint32_t* ids, const float* mean2d,
                                      const float* conic, const float* opacity, const int32_t* topk_idx,
                                      const float* topk_w, const float* dict, const float* pos, int32_t n_neg,
                                      const float* neg, float tau, float* relevancy, void* feat, void* coef,
                                      float* final_T, int32_t* last, void* workspace, size_t workspace_bytes,
                                      hipStream_t stream) {
    if (!pos || !neg || !relevancy || n_neg < 1) return LS2_ERR_ARG;
    if (n_neg > 8) return LS2_ERR_UNSUPPORTED;
    size_t need = 0;
    if (ls2_splat_decode_query_workspace(L, D, n_neg, &need) != LS2_OK) need = 0;  // the shape checks report it
    return splat_decode_query_run(cam, n, levels, K, L, D, tile_ranges, ids, mean2d, conic, opacity, topk_idx, topk_w,
                                  dict, pos, n_neg, neg, tau, relevancy, feat, coef, final_T, last, workspace,
                                  workspace_bytes, need, stream);
}

// ---- ls2_splat_decode_query_noalloc: the same frame with the library's own
// scratch, for callers that cannot allocate (stream capture, serving loops).
//
// The scratch is a fixed device array.  In host code its name only stands in
// for the symbol; the device address of each GPU's copy is looked up once per
// device (hipGetSymbolAddress, with that device current) and only that
// address is passed to kernels.  Every call on a device shares that device's
// copy, so calls that overlap on one GPU race; the repack kernels rewrite
// everything the frame reads on every call, so nothing needs clearing.
constexpr size_t kNoAllocScratchBytes = 160 * 1024;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kNoAllocMaxDevices = 64;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};
std::mutex g_scratch_mu;

void* scratch_ptr() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" int ls2_splat_decode_query_noalloc(const ls2_camera* cam, int32_t n, int32_t levels, int32_t K,
                                              int32_t L, int32_t D, const uint32_t* tile_ranges, const uint32_t* ids,
                                              const float* mean2d, const float* conic, const float* opacity,
                                              const int32_t* topk_idx, const float* topk_w, const float* dict,
                                              const float* pos, int32_t n_neg, const float* neg, float tau,
                                              float* relevancy, void* feat, void* coef, float* final_T,
                                              int32_t* last, hipStream_t stream) {
    if (!pos || !neg || !relevancy || n_neg < 1) return LS2_ERR_ARG;
    if (n_neg > 8) return LS2_ERR_UNSUPPORTED;
    size_t need = 0;
    const int ws = ls2_splat_decode_query_workspace(L, D, n_neg, &need);
    if (ws != LS2_OK) return ws;
    if (need > kNoAllocScratchBytes) return LS2_ERR_CAPACITY;  // before any device call
    void* w = scratch_ptr();
    if (!w) return LS2_ERR_DEVICE;
    return splat_decode_query_run(cam, n, levels, K, L, D, tile_ranges, ids, mean2d, conic, opacity, topk_idx, topk_w,
                                  dict, pos, n_neg, neg, tau, relevancy, feat, coef, final_T, last, w,
                                  kNoAllocScratchBytes, need, stream);
}
