// Lean frame path: the mask pyramid kept as bits and compact arrays.
//
// The blurred mask a_i (Sec. 3.1, Table 1) is positive exactly on the
// Chebyshev dilation of the pooled edges by the blur radius when every
// Gaussian tap is positive and no product of two taps underflows (the host
// checks both), and the nesting step of the inclusive decomposition is then a
// no-op (the host checks the radius condition).  So the stencil of Sec. 4.1
// is computed here as an integer dilation of bit-packed edges, its texels are
// ranked (per-word prefix counts), and a_i and the sub-image values are
// stored only at the stencil texels, indexed by rank.  The merge (Sec. 4.2,
// Eq. 1) finds a texel's value through its rank.  All floating-point results
// are the same operations, in the same order, as the dense path.
#pragma once
#include "eval_common.hpp"

namespace mr {


// horizontal dilation by r (< 32) of word c with neighbours p (left), n (right);
// bit x % 32 of word x / 32 holds texel x
__device__ __forceinline__ unsigned hdilate(unsigned p, unsigned c, unsigned n, int r) {
    unsigned d = c;
    for (int s = 1; s <= r; ++s) d |= (c << s) | (p >> (32 - s)) | (c >> s) | (n << (32 - s));
    return d;
}

__device__ __forceinline__ int lean_level(const LeanArgs& A, unsigned b) {
    int l = 0;
#pragma unroll
    for (int k = 1; k < 3; ++k) l += (k < A.nlev && b >= A.lv[k].blk_base) ? 1 : 0;
    return l;
}

// Words are ranked tile by tile (kLeanTileWords words x kLeanTileRows rows,
// one thread per word, row-major inside a tile, tiles row-major), so that
// consecutive work-list entries lie close together on screen and the
// evaluation's sample gathers of one wave touch a compact region.  The rank
// of a texel is still woff[word] + popcount of the lower bits of its word.
struct TileWord {
    int y, xw;
    bool ok;
    unsigned w;
};

__device__ __forceinline__ TileWord tile_word(const LeanLevel& L, unsigned b, unsigned t) {
    const unsigned bl = b - L.blk_base;
    const unsigned ty = bl / (unsigned)L.tiles_x, tx = bl - ty * (unsigned)L.tiles_x;
    TileWord r;
    r.xw = (int)(tx * kLeanTileWords + (t % kLeanTileWords));
    r.y = (int)(ty * kLeanTileRows + (t / kLeanTileWords));
    r.ok = r.xw < L.wpr && r.y < L.H;
    r.w = (unsigned)r.y * (unsigned)L.wpr + (unsigned)r.xw;
    return r;
}

// Stencil words of one ranking tile (dilated edge bits), separably: the
// tile's edge words plus a halo of R rows and one word on each side are
// staged in LDS, dilated horizontally per row, then ORed over 2R + 1 rows.
// Words outside the level are 0 (no edges), as the blur's zero padding.
constexpr int kStageCols = kLeanTileWords + 2, kStageRows = kLeanTileRows + 2 * kBlurFusedMaxRadiusC;
// Words of a ranking tile: kRankThreads.  The standalone ranking launches run
// one thread per word; the persistent batch launch runs 256-thread blocks,
// two words per thread.  Larger tiles mean fewer list-base atomics on each
// level's counter (1024 ranking blocks of level 1 at 4K with 256-word tiles
// contended for one address).
constexpr int kRankThreads = kLeanTileWords * kLeanTileRows;

// Stencil words of the tile for the NT threads of a block: word
// threadIdx.x + k NT (row-major in the tile) goes to acc[k].
template <int R, int NT>
__device__ __forceinline__ void stencil_tile(const LeanLevel& L, unsigned b, unsigned (*eb)[kStageCols],
                                             unsigned (*hd)[kLeanTileWords], unsigned (&acc)[kRankThreads / NT]) {
    const unsigned bl = b - L.blk_base;
    const unsigned ty = bl / (unsigned)L.tiles_x, tx = bl - ty * (unsigned)L.tiles_x;
    const int yw0 = (int)(ty * kLeanTileRows) - R, xw0 = (int)(tx * kLeanTileWords) - 1;
    constexpr int rows = kLeanTileRows + 2 * R, n = rows * kStageCols;
    // all of a thread's loads are issued before the first LDS store
    constexpr int NI = (n + NT - 1) / NT;
    unsigned v[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int i = threadIdx.x + k * NT;
        const int r = i / kStageCols, c = i - r * kStageCols;
        const int y = yw0 + r, xw = xw0 + c;
        v[k] = (i < n && y >= 0 && y < L.H && xw >= 0 && xw < L.wpr) ? L.Eb[(unsigned)y * (unsigned)L.wpr + (unsigned)xw]
                                                                     : 0u;
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int i = threadIdx.x + k * NT;
        const int r = i / kStageCols, c = i - r * kStageCols;
        if (i < n) eb[r][c] = v[k];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < rows * kLeanTileWords; i += NT) {
        const int r = i / kLeanTileWords, c = i - r * kLeanTileWords;
        hd[r][c] = hdilate(eb[r][c], eb[r][c + 1], eb[r][c + 2], R);
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kRankThreads / NT; ++w) {
        const int t = threadIdx.x + w * NT;
        const int c = t % kLeanTileWords, r0 = t / kLeanTileWords;
        unsigned o = 0;
#pragma unroll
        for (int k = 0; k <= 2 * R; ++k) o |= hd[r0 + k][c];
        acc[w] = o;
    }
}

__device__ __forceinline__ unsigned wave_scan_incl(unsigned v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Ranking, in two launches over the ranking tiles (one block per tile).
//
// 1. k_lean_stencil: the tile's stencil words (dilated edge bits) and the
//    tile's total of stencil texels.
// 2. k_lean_list: the tile's first list position = the sum of the totals of
//    the level's earlier tiles; the rank of every word (woff) and the tile's
//    run of the list.
//
// A level's list holds its tiles' runs in tile order (tiles row-major,
// words row-major inside a tile, bits ascending), so the list is the same on
// every run: a fixed permutation of the row-major list of stencil texels.
// The rank of every texel is stored with it (woff), which is all the merge
// needs.  (A single launch that found each tile's list position by a
// decoupled look-back over the earlier tiles' totals made the ranking about
// 11 us slower at 4K: every tile waited for the slowest of its predecessors.)
template <int NT>
struct StencilLds {
    unsigned wtot[NT / 64];
    unsigned eb[kStageRows][kStageCols];
    unsigned hd[kStageRows][kLeanTileWords];
};

template <int NT>
__device__ __forceinline__ void stencil_block(const LeanArgs& A, unsigned b, StencilLds<NT>& sm) {
    constexpr int WPT = kRankThreads / NT;
    const int l = lean_level(A, b);
    const LeanLevel& L = A.lv[l];
    unsigned acc[WPT] = {};
    switch (L.r) {  // uniform: every thread takes part in the staging
#define MR_STENCIL(R) \
    case R: stencil_tile<R, NT>(L, b, sm.eb, sm.hd, acc); break;
        MR_STENCIL(0) MR_STENCIL(1) MR_STENCIL(2) MR_STENCIL(3) MR_STENCIL(4) MR_STENCIL(5) MR_STENCIL(6)
        MR_STENCIL(7) MR_STENCIL(8)
#undef MR_STENCIL
        default: break;
    }
    unsigned cnt = 0;
#pragma unroll
    for (int w = 0; w < WPT; ++w) {
        const TileWord tw = tile_word(L, b, threadIdx.x + w * NT);
        if (tw.ok) {
            L.Sb[tw.w] = acc[w];
            cnt += __popc(acc[w]);
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d, 64);
    if (__lane_id() == 0) sm.wtot[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned total = 0;
#pragma unroll
        for (int k = 0; k < NT / 64; ++k) total += sm.wtot[k];
        A.tot[b] = total;
    }
}

// A tile of at most kRankStage entries builds its run of the list in LDS
// and stores it with consecutive threads at consecutive positions; the
// entries of a word are kRankStage / 512 = 16 or more dwords apart, so
// storing them straight from each thread would touch a separate cache line
// per thread and entry.  LDS positions are padded by one word per 32, which
// puts the threads' entries in distinct banks.  (Measured at 4K with the
// list built in one launch: 13.3 us with direct stores, 11.5 us staging up
// to 4096 entries, 10.4 us up to 8192.)
constexpr unsigned kRankStage = 8192;
__device__ __forceinline__ unsigned stage_slot(unsigned p) { return p + (p >> 5); }

template <int NT, unsigned STAGE>
struct ListLds {
    unsigned wtot[kRankThreads / 64], wpre[NT / 64];
    unsigned stg[STAGE + STAGE / 32];
};

// Word threadIdx.x + k NT of the tile is the (k NT / 64 + wave)-th run of 64
// words in row-major order, so its exclusive prefix is the totals of the
// earlier runs plus the wave's scan.
template <int NT, unsigned STAGE>
__device__ __forceinline__ void list_block(const LeanArgs& A, unsigned b, ListLds<NT, STAGE>& sm) {
    constexpr int WPT = kRankThreads / NT, NW = NT / 64;
    const int l = lean_level(A, b);
    const LeanLevel& L = A.lv[l];
    TileWord tw[WPT];
    unsigned acc[WPT], cnt[WPT], inc[WPT];
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
        tw[k] = tile_word(L, b, threadIdx.x + k * NT);
        acc[k] = tw[k].ok ? L.Sb[tw[k].w] : 0u;
    }
    // the level's earlier tiles: their totals summed by the block
    unsigned pre = 0;
    for (unsigned u = L.blk_base + threadIdx.x; u < b; u += NT) pre += A.tot[u];
    const unsigned total = A.tot[b];
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
        cnt[k] = __popc(acc[k]);
        inc[k] = wave_scan_incl(cnt[k]);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) pre += __shfl_xor(pre, d, 64);
    const int wv = threadIdx.x >> 6;
    if (__lane_id() == 63) {
#pragma unroll
        for (int k = 0; k < WPT; ++k) sm.wtot[k * NW + wv] = inc[k];
    }
    if (__lane_id() == 0) sm.wpre[wv] = pre;
    __syncthreads();
    unsigned tb = 0;  // entries of the level before this tile
#pragma unroll
    for (int k = 0; k < NW; ++k) tb += sm.wpre[k];
    unsigned ex[WPT];  // entries of the tile before each word
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
        ex[k] = inc[k] - cnt[k];
        const int run = k * NW + wv;
#pragma unroll
        for (int j = 0; j < kRankThreads / 64; ++j) ex[k] += j < run ? sm.wtot[j] : 0u;
        if (tw[k].ok) L.woff[tw[k].w] = tb + ex[k];
    }
    if (threadIdx.x == 0 && b == L.blk_base + L.ntiles - 1) A.count[L.count_idx] = tb + total;
    if (total > STAGE) {  // uniform
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const unsigned base = (unsigned)tw[k].y * (unsigned)L.W + (unsigned)tw[k].xw * 32u;
            unsigned m = acc[k], pos = tb + ex[k];  // m = 0 outside the level
            while (m) {
                const int bit = __builtin_ctz(m);
                m &= m - 1;
                L.list[pos++] = base + (unsigned)bit;
            }
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
        const unsigned base = (unsigned)tw[k].y * (unsigned)L.W + (unsigned)tw[k].xw * 32u;
        unsigned m = acc[k], q = ex[k];
        while (m) {
            const int bit = __builtin_ctz(m);
            m &= m - 1;
            sm.stg[stage_slot(q++)] = base + (unsigned)bit;
        }
    }
    __syncthreads();
    for (unsigned j = threadIdx.x; j < total; j += NT) L.list[tb + j] = sm.stg[stage_slot(j)];
}

// ---------------------------------------------------------------------------
// merge with rank lookups (same arithmetic as the dense merge)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void axis_taps_l(int X, int sh, int n, int lo, int& ia, int& ib, float& f) {
    const int s = 1 << sh;
    const int m = X - (s >> 1);
    const int x0 = m >> sh;
    f = ((float)(m & (s - 1)) + 0.5f) * (1.0f / (float)s);
    ia = min(max(x0, 0), n - 1) - lo;
    ib = min(max(x0 + 1, 0), n - 1) - lo;
}

// value of a sub-image (f32 or f16 storage)
template <typename VT>
__device__ __forceinline__ float cval(const void* c, long long i) {
    return (float)static_cast<const VT*>(c)[i];
}

template <int C>
struct MergeLds {
    float la[kMergeLDS];
    uint8_t ls[kMergeLDS];
    float lc[C][kMergeLDS];
    int lvl_any[kMaxLevels];  // some staged a > 0 in the level's region
};

template <int C, typename VT>
__device__ __forceinline__ void merge_tile(const LeanMergeArgs& a, unsigned tile, unsigned tiles_x, float* la,
                                           uint8_t* ls, float (*lc)[kMergeLDS], int* lvl_any) {
    const int x0 = (int)(tile % tiles_x) * kMergeTW;
    const int y0 = (int)(tile / tiles_x) * kMergeTH;
    const int nl = a.nlev, t = threadIdx.x;
    if (t < kMaxLevels) lvl_any[t] = 0;
    __syncthreads();
    // ---- stage the coarse levels' tap regions (all loads issued first) ----
    constexpr int kSlots = (kMergeLDS + 255) / 256;
    uint8_t sv[kSlots];
    float av[kSlots], cv[kSlots][C];
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
        const int idx = t + 256 * j;
        sv[j] = 0;
        av[j] = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) cv[j][c] = 0.0f;
        if (idx >= a.staged) continue;
        int q = 0;
#pragma unroll
        for (int k = 1; k < kMaxLevels; ++k) q += (k < nl && idx >= a.lv[k].roff) ? 1 : 0;
        // the levels' regions start at multiples of 64 slots: one level per wave
        q = __builtin_amdgcn_readfirstlane(q);
        const LeanMergeLevel& L = a.lv[q];
        const int k = idx - L.roff;
        if (k >= L.rw * L.rh) continue;  // padding of the level's region
        const int yy = (int)(((unsigned)k * L.rmagic) >> 16), xx = k - yy * L.rw;
        const int Xl = min(max((x0 >> L.sh) - 1 + xx, 0), L.W - 1);
        const int Yl = min(max((y0 >> L.sh) - 1 + yy, 0), L.H - 1);
        if (q == nl - 1) {
            sv[j] = 1;
            const unsigned p = (unsigned)Yl * (unsigned)L.W + (unsigned)Xl;
#pragma unroll
            for (int c = 0; c < C; ++c) cv[j][c] = cval<VT>(L.c, c * L.c_plane + p);
        } else {
            const unsigned wi = (unsigned)Yl * (unsigned)L.wpr + (unsigned)(Xl >> 5);
            const unsigned word = L.Sb[wi];
            const unsigned bit = (unsigned)Xl & 31u;
            if ((word >> bit) & 1u) {
                const unsigned rank = L.woff[wi] + __popc(word & ((1u << bit) - 1u));
                sv[j] = 1;
                av[j] = L.ac[rank];
#pragma unroll
                for (int c = 0; c < C; ++c) cv[j][c] = cval<VT>(L.c, c * L.c_plane + rank);
            }
        }
    }
    const int q = t & 15, row = t >> 4;
    const int Y = y0 + row;
    const int XQ = x0 + 4 * q;
    const bool active = Y < a.H && XQ < a.W;
    // ---- level 1: four pixels per thread, values by rank ----
    uint8_t s1[4] = {0, 0, 0, 0};
    float a1[4] = {0, 0, 0, 0}, c1[C][4];
#pragma unroll
    for (int c = 0; c < C; ++c) c1[c][0] = c1[c][1] = c1[c][2] = c1[c][3] = 0.0f;
    const bool fine1 = a.fine1;
    if (fine1 && active) {
        const LeanMergeLevel& L = a.lv[0];
        const unsigned wi = (unsigned)Y * (unsigned)L.wpr + (unsigned)(XQ >> 5);
        const unsigned word = L.Sb[wi];
        const unsigned bit = (unsigned)XQ & 31u;
        const unsigned nib = (word >> bit) & 0xFu;
        if (nib) {
            unsigned rank = L.woff[wi] + __popc(word & ((1u << bit) - 1u));
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if ((nib >> k) & 1u) {
                    s1[k] = 1;
                    a1[k] = L.ac[rank];
#pragma unroll
                    for (int c = 0; c < C; ++c) c1[c][k] = cval<VT>(L.c, c * L.c_plane + rank);
                    ++rank;
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
        const int idx = t + 256 * j;
        if (idx >= a.staged) continue;
        ls[idx] = sv[j];
        la[idx] = av[j];
#pragma unroll
        for (int c = 0; c < C; ++c) lc[c][idx] = cv[j][c];
        if (av[j] != 0.0f) {
            int q = 0;
#pragma unroll
            for (int k = 1; k < kMaxLevels; ++k) q += (k < nl && idx >= a.lv[k].roff) ? 1 : 0;
            lvl_any[q] = 1;
        }
    }
    __syncthreads();
    if (!active) return;

    float out[C][4];
    {
        // coarsest level: plain bilinear, normalising sum exactly 1
        const LeanMergeLevel& L = a.lv[nl - 1];
        int ya, yb;
        float fy;
        axis_taps_l(Y, L.sh, L.H, (y0 >> L.sh) - 1, ya, yb, fy);
        const float gy = 1.0f - fy;
        const int r0 = L.roff + ya * L.rw, r1 = L.roff + yb * L.rw;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int xa, xb;
            float fx;
            axis_taps_l(XQ + k, L.sh, L.W, (x0 >> L.sh) - 1, xa, xb, fx);
            const float gx = 1.0f - fx;
            const float b0 = gx * gy, b1 = fx * gy, b2 = gx * fy, b3 = fx * fy;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float num = b0 * lc[c][r0 + xa];
                num = num + b1 * lc[c][r0 + xb];
                num = num + b2 * lc[c][r1 + xa];
                num = num + b3 * lc[c][r1 + xb];
                out[c][k] = num;
            }
        }
    }
    for (int j = nl - 2; j >= 0; --j) {
        const LeanMergeLevel& L = a.lv[j];
        if (j == 0 && fine1) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool in = s1[k] != 0;
                const float alpha = in ? fminf(a1[k] * L.w, 1.0f) : 0.0f;
                const float om = 1.0f - alpha;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const float Ci = in ? c1[c][k] : 0.0f;
                    out[c][k] = Ci * alpha + out[c][k] * om;
                }
            }
            continue;
        }
        // every staged a of this level is 0: A = 0 at all pixels, alpha = 0
        if (!lvl_any[j]) continue;
        int ya, yb;
        float fy;
        axis_taps_l(Y, L.sh, L.H, (y0 >> L.sh) - 1, ya, yb, fy);
        const float gy = 1.0f - fy;
        const int r0 = L.roff + ya * L.rw, r1 = L.roff + yb * L.rw;
        float A[4], b[4][4];
        int ix[4][2];
        bool nz = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int xa, xb;
            float fx;
            axis_taps_l(XQ + k, L.sh, L.W, (x0 >> L.sh) - 1, xa, xb, fx);
            const float gx = 1.0f - fx;
            b[k][0] = gx * gy;
            b[k][1] = fx * gy;
            b[k][2] = gx * fy;
            b[k][3] = fx * fy;
            ix[k][0] = xa;
            ix[k][1] = xb;
            float s_ = b[k][0] * la[r0 + xa];
            s_ = s_ + b[k][1] * la[r0 + xb];
            s_ = s_ + b[k][2] * la[r1 + xa];
            s_ = s_ + b[k][3] * la[r1 + xb];
            A[k] = s_;
            nz |= s_ != 0.0f;
        }
        if (!nz) continue;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i00 = r0 + ix[k][0], i01 = r0 + ix[k][1], i10 = r1 + ix[k][0], i11 = r1 + ix[k][1];
            const bool e0 = ls[i00] != 0, e1 = ls[i01] != 0, e2 = ls[i10] != 0, e3 = ls[i11] != 0;
            float den = e0 ? b[k][0] : 0.0f;
            den = den + (e1 ? b[k][1] : 0.0f);
            den = den + (e2 ? b[k][2] : 0.0f);
            den = den + (e3 ? b[k][3] : 0.0f);
            const bool use = A[k] != 0.0f && den > 0.0f;
            const float alpha = use ? fminf(A[k] * L.w, 1.0f) : 0.0f;
            const float om = 1.0f - alpha;
            const float dd = use ? den : 1.0f;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float num = e0 ? b[k][0] * lc[c][i00] : 0.0f;
                num = num + (e1 ? b[k][1] * lc[c][i01] : 0.0f);
                num = num + (e2 ? b[k][2] * lc[c][i10] : 0.0f);
                num = num + (e3 ? b[k][3] * lc[c][i11] : 0.0f);
                const float Ci = use ? (dd == 1.0f ? num : num / dd) : 0.0f;
                out[c][k] = Ci * alpha + out[c][k] * om;
            }
        }
    }
    const unsigned p = (unsigned)Y * (unsigned)a.W + (unsigned)XQ;
    const unsigned plane = (unsigned)a.W * (unsigned)a.H;
#pragma unroll
    for (int c = 0; c < C; ++c)
        store_stream4(a.out + c * plane + p, out[c][0], out[c][1], out[c][2], out[c][3]);
}

// ---------------------------------------------------------------------------
// merge for the four consecutive levels 1, 2, 3, 4 (scales 1, 2, 4, 8): the
// same arithmetic as k_lean_merge with the tap geometry fixed at compile
// time.  A thread's four pixels start at a multiple of 4, so for scales 2 and
// 4 their tap phases (fx) and column offsets are constants; a level's values
// are staged once per tile, stencil membership is a > 0 (exact on this path)
// and texels off the stencil are staged as 0, so that their products with
// the tap weights are +0 and leave the sums unchanged.
// ---------------------------------------------------------------------------
template <int SH>
__device__ __forceinline__ void taps4(int X, int n, int lo, int& ia, int& ib, float& f) {
    constexpr int s = 1 << SH;
    const int m = X - (s >> 1);
    const int x0 = m >> SH;
    f = ((float)(m & (s - 1)) + 0.5f) * (1.0f / (float)s);
    ia = min(max(x0, 0), n - 1) - lo;
    ib = min(max(x0 + 1, 0), n - 1) - lo;
}

// The x taps of a thread's four pixels X = XQ + k (XQ a multiple of 4) at
// scale s = 2^SH, with m = X - s/2, x0 = m >> SH, fx = ((m & (s-1)) + 0.5)/s:
//   s = 2: k = 0..3 -> x0 = XQ/2 - 1, XQ/2, XQ/2, XQ/2 + 1; fx = 3/4, 1/4, 3/4, 1/4
//   s = 4: x0 = XQ/4 - 1, XQ/4 - 1, XQ/4, XQ/4; fx = 5/8, 7/8, 1/8, 3/8
//   s = 8: x0 = XQ/8 - 1 (all k) and fx = (4.5 + k)/8 when XQ % 8 = 0,
//          x0 = XQ/8 and fx = (0.5 + k)/8 when XQ % 8 = 4.
// So the four pixels read at most 4 distinct tap columns: col[j] = x-tap
// base + j (clamped to the level, relative to the staged region), and
// pixel k uses columns cofs(k) and cofs(k) + 1.
template <int SH>
struct XTaps4 {
    static constexpr int ncol = SH == 1 ? 4 : (SH == 2 ? 3 : 2);
    __device__ static constexpr int cofs(int k) { return SH == 1 ? (k + 1) / 2 : (SH == 2 ? k / 2 : 0); }
    __device__ static float fx(int k, int XQ) {
        if (SH == 1) return (k & 1) ? 0.25f : 0.75f;
        if (SH == 2) return (float)(2 * ((k + 2) & 3) + 1) * 0.125f;
        return (XQ & 4) ? (0.5f + (float)k) * 0.125f : (4.5f + (float)k) * 0.125f;
    }
    // first tap column (level texels, before clamping)
    __device__ static int base(int XQ) { return SH == 3 ? ((XQ & 4) ? XQ >> 3 : (XQ >> 3) - 1) : (XQ >> SH) - 1; }
};

// staged region of a level: (kMergeTW >> SH) + 2 columns, (kMergeTH >> SH) + 2 rows
template <int SH>
struct Region4 {
    static constexpr int rw = (kMergeTW >> SH) + 2, rh = (kMergeTH >> SH) + 2, n = rw * rh;
};

// one list level (scale 2^SH) blended into out[][4] for the thread's pixels
template <int SH, int C>
__device__ __forceinline__ void blend4(const float* la, const float (*lc)[Region4<SH>::n], const LeanMergeLevel& L,
                                       int x0, int y0, int XQ, int Y, float (&out)[C][4]) {
    using XT = XTaps4<SH>;
    constexpr int RW = Region4<SH>::rw;
    int ya, yb;
    float fy;
    taps4<SH>(Y, L.H, (y0 >> SH) - 1, ya, yb, fy);
    const float gy = 1.0f - fy;
    const int r0 = ya * RW, r1 = yb * RW;
    const int lo = (x0 >> SH) - 1, xb0 = XT::base(XQ);
    int col[XT::ncol];
    float a0[XT::ncol], a1[XT::ncol];
#pragma unroll
    for (int j = 0; j < XT::ncol; ++j) {
        col[j] = min(max(xb0 + j, 0), L.W - 1) - lo;
        a0[j] = la[r0 + col[j]];
        a1[j] = la[r1 + col[j]];
    }
    // a >= 0 and every tap weight > 0, so A = 0 at all four pixels (alpha = 0,
    // out unchanged) exactly when all their tap values are +0
    unsigned any = 0u;
#pragma unroll
    for (int j = 0; j < XT::ncol; ++j) any |= __float_as_uint(a0[j]) | __float_as_uint(a1[j]);
    if (!any) return;
    float A[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int ja = XT::cofs(k), jb = ja + 1;
        const float fx = XT::fx(k, XQ), gx = 1.0f - fx;
        float s_ = (gx * gy) * a0[ja];
        s_ = s_ + (fx * gy) * a0[jb];
        s_ = s_ + (gx * fy) * a1[ja];
        s_ = s_ + (fx * fy) * a1[jb];
        A[k] = s_;
    }
    float v0[C][XT::ncol], v1[C][XT::ncol];
#pragma unroll
    for (int j = 0; j < XT::ncol; ++j)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            v0[c][j] = lc[c][r0 + col[j]];
            v1[c][j] = lc[c][r1 + col[j]];
        }
    // C_i = num / den, with the division only where a tap lies off the
    // stencil (den < 1); a wave whose pixels all have den = 1 skips it
    float Ci[C][4], alpha[4], den[4];
    bool part[4], need = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int ja = XT::cofs(k), jb = ja + 1;
        const float fx = XT::fx(k, XQ), gx = 1.0f - fx;
        const float b0 = gx * gy, b1 = fx * gy, b2 = gx * fy, b3 = fx * fy;
        float d = a0[ja] > 0.0f ? b0 : 0.0f;
        d = d + (a0[jb] > 0.0f ? b1 : 0.0f);
        d = d + (a1[ja] > 0.0f ? b2 : 0.0f);
        d = d + (a1[jb] > 0.0f ? b3 : 0.0f);
        const bool use = A[k] != 0.0f && d > 0.0f;
        alpha[k] = use ? fminf(A[k] * L.w, 1.0f) : 0.0f;
        den[k] = d;
        part[k] = use && d != 1.0f;
        need = need || part[k];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            float num = b0 * v0[c][ja];
            num = num + b1 * v0[c][jb];
            num = num + b2 * v1[c][ja];
            num = num + b3 * v1[c][jb];
            Ci[c][k] = use ? num : 0.0f;
        }
    }
    if (__ballot(need)) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (part[k]) Ci[c][k] = Ci[c][k] / den[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float om = 1.0f - alpha[k];
#pragma unroll
        for (int c = 0; c < C; ++c) out[c][k] = Ci[c][k] * alpha[k] + out[c][k] * om;
    }
}

// one staged texel: index k of the (kMergeTW >> SH) + 2 columns wide region
// of the level in argument slot LV (scale 2^SH) around the tile at (x0, y0),
// clamped to the level; DENSE: the coarsest level, read densely, the others
// by rank (a = 0 and values 0 off the stencil)
template <int LV, int SH, int RW, int C, typename VT, bool DENSE = LV == 3>
__device__ __forceinline__ void stage4(const LeanMergeArgs& a, int k, int x0, int y0, float& av, float (&cv)[C]) {
    const LeanMergeLevel& L = a.lv[LV];
    const int yy = k / RW, xx = k - yy * RW;
    const int Xl = min(max((x0 >> SH) - 1 + xx, 0), L.W - 1);
    const int Yl = min(max((y0 >> SH) - 1 + yy, 0), L.H - 1);
    av = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) cv[c] = 0.0f;
    if (DENSE) {
        const unsigned p = (unsigned)Yl * (unsigned)L.W + (unsigned)Xl;
#pragma unroll
        for (int c = 0; c < C; ++c) cv[c] = cval<VT>(L.c, c * L.c_plane + p);
    } else {
        const unsigned wi = (unsigned)Yl * (unsigned)L.wpr + (unsigned)(Xl >> 5);
        const unsigned word = L.Sb[wi];
        const unsigned bit = (unsigned)Xl & 31u;
        if ((word >> bit) & 1u) {
            const unsigned rank = L.woff[wi] + __popc(word & ((1u << bit) - 1u));
            av = L.ac[rank];
#pragma unroll
            for (int c = 0; c < C; ++c) cv[c] = cval<VT>(L.c, c * L.c_plane + rank);
        }
    }
}

template <int C>
struct Merge4Lds {
    float la2[Region4<1>::n], la3[Region4<2>::n];
    float lc2[C][Region4<1>::n], lc3[C][Region4<2>::n], lc4[C][Region4<3>::n];
    int any2, any3;
};

// L2 false: the levels 1, 3 and 4 (SSGI's Table 1 column), in argument
// slots 0, 1 and 2: the same merge without level 2's staging and blend.
template <int C, typename VT, bool L2 = true>
__device__ __forceinline__ void merge4_tile(const LeanMergeArgs& a, unsigned tile, unsigned tiles_x,
                                            Merge4Lds<C>& sm) {
    constexpr int I3 = L2 ? 2 : 1, I4 = L2 ? 3 : 2;  // argument slots of levels 3 and 4
    using R2 = Region4<1>;
    using R3 = Region4<2>;
    using R4 = Region4<3>;
    float* la2 = sm.la2;
    float* la3 = sm.la3;
    float (*lc2)[R2::n] = sm.lc2;
    float (*lc3)[R3::n] = sm.lc3;
    float (*lc4)[R4::n] = sm.lc4;
    int& any2 = sm.any2;
    int& any3 = sm.any3;
    const int x0 = (int)(tile % tiles_x) * kMergeTW;
    const int y0 = (int)(tile / tiles_x) * kMergeTH;
    const int t = threadIdx.x;
    if (t == 0) any2 = any3 = 0;
    __syncthreads();
    // ---- stage levels 2, 3 (by rank, 0 off the stencil) and 4 (dense) ----
    // Every thread stages texel t of level 2 and at most one more: level 2's
    // remaining texels on threads [0, nB), level 4 on [nB, nB + n4), level 3
    // on [128, 128 + n3).  Each slot's level is fixed at compile time, so its
    // parameters are scalar and its divisions by the region width constant.
    // Without level 2: level 4 on threads [0, n4), level 3 on [128, 128 + n3).
    constexpr int nB = R2::n - 256;
    constexpr int n4lo = L2 ? nB : 0;  // first thread staging level 4
    static_assert(nB > 0 && nB + R4::n <= 128 && 128 + R3::n <= 256, "merge staging layout");
    float av[2], cv[2][C];
    av[0] = av[1] = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) cv[0][c] = cv[1][c] = 0.0f;
    if constexpr (L2) stage4<1, 1, R2::rw, C, VT>(a, t, x0, y0, av[0], cv[0]);
    if (L2 && t < nB)
        stage4<1, 1, R2::rw, C, VT>(a, 256 + t, x0, y0, av[1], cv[1]);
    else if (t >= n4lo && t < n4lo + R4::n)
        stage4<I4, 3, R4::rw, C, VT, true>(a, t - n4lo, x0, y0, av[1], cv[1]);
    else if (t >= 128 && t < 128 + R3::n)
        stage4<I3, 2, R3::rw, C, VT, false>(a, t - 128, x0, y0, av[1], cv[1]);
    // a wave covers a 16 x 16 pixel square of the tile (four pixels of a row
    // per thread), so that the pixels near a stencil, where the blends run,
    // fill fewer waves
    const int w = t >> 6, l = t & 63;
    const int Y = y0 + (l >> 2);
    const int XQ = x0 + 16 * w + 4 * (l & 3);
    const bool active = Y < a.H && XQ < a.W;
    // ---- level 1: four pixels per thread, values by rank ----
    float a1[4] = {0, 0, 0, 0}, c1[C][4];
    unsigned nib = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) c1[c][0] = c1[c][1] = c1[c][2] = c1[c][3] = 0.0f;
    if (active) {
        const LeanMergeLevel& L = a.lv[0];
        const unsigned wi = (unsigned)Y * (unsigned)L.wpr + (unsigned)(XQ >> 5);
        const unsigned word = L.Sb[wi];
        const unsigned bit = (unsigned)XQ & 31u;
        nib = (word >> bit) & 0xFu;
        if (nib) {
            unsigned rank = L.woff[wi] + __popc(word & ((1u << bit) - 1u));
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if ((nib >> k) & 1u) {
                    a1[k] = L.ac[rank];
#pragma unroll
                    for (int c = 0; c < C; ++c) c1[c][k] = cval<VT>(L.c, c * L.c_plane + rank);
                    ++rank;
                }
            }
        }
    }
    bool nz2 = false, nz3 = false;
    if constexpr (L2) {
        la2[t] = av[0];
#pragma unroll
        for (int c = 0; c < C; ++c) lc2[c][t] = cv[0][c];
        nz2 = av[0] != 0.0f;
    }
    if (L2 && t < nB) {
        la2[256 + t] = av[1];
#pragma unroll
        for (int c = 0; c < C; ++c) lc2[c][256 + t] = cv[1][c];
        nz2 = nz2 || av[1] != 0.0f;
    } else if (t >= n4lo && t < n4lo + R4::n) {
#pragma unroll
        for (int c = 0; c < C; ++c) lc4[c][t - n4lo] = cv[1][c];
    } else if (t >= 128 && t < 128 + R3::n) {
        la3[t - 128] = av[1];
#pragma unroll
        for (int c = 0; c < C; ++c) lc3[c][t - 128] = cv[1][c];
        nz3 = av[1] != 0.0f;
    }
    if (nz2) any2 = 1;
    if (nz3) any3 = 1;
    __syncthreads();
    if (!active) return;

    float out[C][4];
    {
        // coarsest level (scale 8): plain bilinear, normalising sum exactly 1
        using XT = XTaps4<3>;
        const LeanMergeLevel& L = a.lv[I4];
        int ya, yb;
        float fy;
        taps4<3>(Y, L.H, (y0 >> 3) - 1, ya, yb, fy);
        const float gy = 1.0f - fy;
        const int r0 = ya * R4::rw, r1 = yb * R4::rw;
        const int lo = (x0 >> 3) - 1, xb0 = XT::base(XQ);
        const int ca = min(max(xb0, 0), L.W - 1) - lo, cb = min(max(xb0 + 1, 0), L.W - 1) - lo;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float v00 = lc4[c][r0 + ca], v01 = lc4[c][r0 + cb], v10 = lc4[c][r1 + ca], v11 = lc4[c][r1 + cb];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float fx = XT::fx(k, XQ), gx = 1.0f - fx;
                float num = (gx * gy) * v00;
                num = num + (fx * gy) * v01;
                num = num + (gx * fy) * v10;
                num = num + (fx * fy) * v11;
                out[c][k] = num;
            }
        }
    }
    if (any3) blend4<2, C>(la3, lc3, a.lv[I3], x0, y0, XQ, Y, out);
    if (L2 && any2) blend4<1, C>(la2, lc2, a.lv[1], x0, y0, XQ, Y, out);
    if (nib) {
        const float w1 = a.lv[0].w;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!((nib >> k) & 1u)) continue;  // alpha_1 = 0: out unchanged
            const float alpha = fminf(a1[k] * w1, 1.0f);
            const float om = 1.0f - alpha;
#pragma unroll
            for (int c = 0; c < C; ++c) out[c][k] = c1[c][k] * alpha + out[c][k] * om;
        }
    }
    const unsigned p = (unsigned)Y * (unsigned)a.W + (unsigned)XQ;
    const unsigned plane = (unsigned)a.W * (unsigned)a.H;
#pragma unroll
    for (int c = 0; c < C; ++c)
        store_stream4(a.out + c * plane + p, out[c][0], out[c][1], out[c][2], out[c][3]);
}

}  // namespace mr
