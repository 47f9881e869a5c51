// Bilateral blur of SSAO sub-images (Sec. 4.1) on the compact frame path.
//
// One thread per rendered texel of every blurred level, the levels' item
// ranges padded to whole waves so that a wave's level is uniform.  A tap's
// value is found from the stencil bits: its rank is the rank of its stencil
// word's first texel plus the set bits before it, so values stay stored by
// rank and the merge reads the blurred values exactly where it read the
// unblurred ones.  Taps outside the level, outside the stencil, with invalid
// depth or with a range weight that is not positive add w = +0 (times a
// finite value) to both sums, which leaves them bit-identical to sums over
// the taking-part taps alone in window order.
#include "eval_common.hpp"

namespace mr {
namespace {

struct BilateralMap {
    unsigned cum[kMaxLevels + 1];
    int nlev;
};

__device__ __forceinline__ BilateralMap bilateral_map(const BilateralArgs& a) {
    BilateralMap m;
    m.nlev = a.nlev;
    m.cum[0] = 0;
#pragma unroll
    for (int j = 0; j < kMaxLevels; ++j) {
        unsigned n = 0;
        if (j < a.nlev) n = a.lv[j].list ? min(a.counts[a.lv[j].count_idx], a.lv[j].dense_n) : a.lv[j].dense_n;
        m.cum[j + 1] = m.cum[j] + ((n + 63u) & ~63u);
    }
    return m;
}

template <int R, typename VT>
__device__ __forceinline__ void bilateral_item(const BilateralArgs& a, const BilateralMap& m, unsigned item) {
    int j = 0;
#pragma unroll
    for (int k = 1; k < kMaxLevels; ++k) j += (k < m.nlev && item >= m.cum[k]) ? 1 : 0;
    j = __builtin_amdgcn_readfirstlane(j);
    const BilateralLevel& L = a.lv[j];
    const unsigned local = item - m.cum[j];
    const unsigned n = L.list ? min(a.counts[L.count_idx], L.dense_n) : L.dense_n;
    if (local >= n) return;  // padding of the level's item range
    const unsigned t = L.list ? L.list[local] : local;
    if (t >= L.dense_n) return;  // malformed list entry
    const int y = (int)(t / (unsigned)L.W), x = (int)(t - (unsigned)y * (unsigned)L.W);
    const unsigned own = L.list ? local : t;
    const VT* c = static_cast<const VT*>(L.c);
    const float zp = L.z[t];
    float res = static_cast<float>(c[own]);
    if (valid_depth(zp)) {
        const float d = a.drel * zp;
        // Branch-free window: every tap loads (a tap that does not take part
        // reads the centre texel) and takes weight +0, which leaves both sums
        // unchanged, so all loads of a row can be in flight together.  The
        // window spans at most two stencil words per row (R < 32).
        constexpr int N = 2 * R + 1;
        const int wa = max(x - R, 0) >> 5, wz_ = min(x + R, L.W - 1) >> 5;
        unsigned sb[N][2], so[N][2];
        if (L.list) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int qy = min(max(y - R + k, 0), L.H - 1);
                const unsigned r0 = (unsigned)qy * (unsigned)L.wpr;
                sb[k][0] = L.Sb[r0 + (unsigned)wa];
                sb[k][1] = L.Sb[r0 + (unsigned)wz_];
                so[k][0] = L.woff[r0 + (unsigned)wa];
                so[k][1] = L.woff[r0 + (unsigned)wz_];
            }
        }
        float num = 0.0f, den = 0.0f;
#pragma unroll
        for (int dy = -R; dy <= R; ++dy) {
            const int qy = y + dy;
            const bool rok = qy >= 0 && qy < L.H;
#pragma unroll
            for (int dx = -R; dx <= R; ++dx) {
                const int qx = x + dx;
                bool ok = rok && qx >= 0 && qx < L.W;
                const unsigned qt = ok ? (unsigned)qy * (unsigned)L.W + (unsigned)qx : t;
                unsigned qo = qt;
                if (L.list) {
                    const int h = ((unsigned)qx >> 5) == (unsigned)wa ? 0 : 1;
                    const unsigned bits = sb[dy + R][h], b = (unsigned)qx & 31u;
                    ok = ok && ((bits >> b) & 1u);
                    qo = so[dy + R][h] + (unsigned)__popc(bits & ((1u << b) - 1u));
                }
                qo = ok ? qo : own;
                const float zq = L.z[ok ? qt : t];
                const float v = static_cast<float>(c[qo]);
                const float wz = 1.0f - fabsf(zq - zp) / d;
                ok = ok && valid_depth(zq) && wz > 0.0f;
                const float w = ok ? (a.wb[dy + R] * a.wb[dx + R]) * wz : 0.0f;
                num = num + w * v;
                den = den + w;
            }
        }
        res = num / den;
    }
    static_cast<VT*>(L.out)[own] = static_cast<VT>(res);
}

template <int R, typename VT>
__global__ __launch_bounds__(256) void k_bilateral(BilateralArgs a) {
    const BilateralMap m = bilateral_map(a);
    const ChunkRange cr = chunk_range((m.cum[kMaxLevels] + 255u) / 256u);
    for (unsigned ch = cr.first; ch < cr.end; ch += cr.step) {
        const unsigned item = ch * 256u + threadIdx.x;
        if (item < m.cum[kMaxLevels]) bilateral_item<R, VT>(a, m, item);
    }
}

}  // namespace

hipError_t launch_bilateral(const BilateralArgs& a, unsigned total_hint, hipStream_t s) {
#define MR_BL(R, VT) \
    hipLaunchKernelGGL((k_bilateral<R, VT>), dim3(eval_blocks<k_bilateral<R, VT>>(total_hint)), dim3(256), 0, s, a)
    if (a.R == 1) {
        if (a.c16) MR_BL(1, _Float16);
        else MR_BL(1, float);
    } else {
        if (a.c16) MR_BL(2, _Float16);
        else MR_BL(2, float);
    }
#undef MR_BL
    return hipGetLastError();
}

}  // namespace mr
