// Work-list compaction: the stencil test of Sec. 4.1 turned into per-level
// lists of the texels to evaluate, in row-major ascending order, with the
// list lengths left on the device.
//
// Three passes over the stencils of all compacted levels at once (a level's
// stencil is cut into chunks of 4096 texels, 16 per thread):
//   count   - nonzero bytes per chunk (popcount of a byte mask, block sum);
//   scan    - one workgroup turns chunk counts into chunk offsets per level
//             and writes the level totals;
//   scatter - each chunk recounts, takes a wave64 prefix sum of the per-thread
//             counts plus the wave totals from LDS, and writes its indices.
#include "mr_internal.hpp"

namespace mr {

// number of nonzero bytes of a 32-bit word
__device__ __forceinline__ unsigned nz_bytes(unsigned w) {
    return __popc((((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) & 0x80808080u);
}

__device__ __forceinline__ int find_level(const CompactArgs& a, unsigned c) {
    int l = 0;
    while (l + 1 < a.nlev && c >= a.chunk_base[l + 1]) ++l;
    return l;
}

// 16 stencil bytes of one thread (bytes past the end read as 0)
__device__ __forceinline__ uint4 load16(const uint8_t* S, unsigned n, unsigned off) {
    if (off + 16 <= n) return *reinterpret_cast<const uint4*>(S + off);
    unsigned w[4] = {0, 0, 0, 0};
    for (unsigned b = 0; b < 16 && off + b < n; ++b) w[b >> 2] |= (unsigned)S[off + b] << (8 * (b & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ unsigned wave_incl_scan(unsigned v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        unsigned o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

__global__ __launch_bounds__(256) void k_count(CompactArgs a) {
    __shared__ unsigned wsum[4];
    const unsigned c = blockIdx.x;
    const int l = find_level(a, c);
    const unsigned off = (c - a.chunk_base[l]) * kChunk + threadIdx.x * 16;
    unsigned cnt = 0;
    if (off < a.n[l]) {
        const uint4 v = load16(a.S[l], a.n[l], off);
        cnt = nz_bytes(v.x) + nz_bytes(v.y) + nz_bytes(v.z) + nz_bytes(v.w);
    }
    // wave reduction
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d, 64);
    if (__lane_id() == 0) wsum[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) a.chunk_count[c] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ __launch_bounds__(1024) void k_scan(CompactArgs a) {
    __shared__ unsigned wtot[16];
    const int t = threadIdx.x, lane = __lane_id(), wv = t >> 6;
    // levels that are not compacted report 0
    if (t < kMaxLevels) a.count[t] = 0;
    __syncthreads();
    for (int l = 0; l < a.nlev; ++l) {
        const unsigned b0 = a.chunk_base[l], b1 = a.chunk_base[l + 1];
        unsigned carry = 0;
        for (unsigned base = b0; base < b1; base += 1024) {
            const unsigned c = base + t;
            const unsigned v = c < b1 ? a.chunk_count[c] : 0u;
            const unsigned inc = wave_incl_scan(v);
            if (lane == 63) wtot[wv] = inc;
            __syncthreads();
            unsigned before = 0, all = 0;
            for (int w = 0; w < 16; ++w) {
                if (w < wv) before += wtot[w];
                all += wtot[w];
            }
            if (c < b1) a.chunk_off[c] = carry + before + inc - v;
            carry += all;
            __syncthreads();
        }
        if (t == 0) a.count[a.count_idx[l]] = carry;
    }
}

__global__ __launch_bounds__(256) void k_scatter(CompactArgs a) {
    __shared__ unsigned wtot[4];
    const unsigned c = blockIdx.x;
    const int l = find_level(a, c);
    const unsigned base = (c - a.chunk_base[l]) * kChunk;
    const unsigned off = base + threadIdx.x * 16;
    uint4 v = make_uint4(0, 0, 0, 0);
    unsigned cnt = 0;
    if (off < a.n[l]) {
        v = load16(a.S[l], a.n[l], off);
        cnt = nz_bytes(v.x) + nz_bytes(v.y) + nz_bytes(v.z) + nz_bytes(v.w);
    }
    const unsigned inc = wave_incl_scan(cnt);
    const int wv = threadIdx.x >> 6;
    if (__lane_id() == 63) wtot[wv] = inc;
    __syncthreads();
    unsigned before = 0;
    for (int w = 0; w < wv; ++w) before += wtot[w];
    unsigned pos = a.chunk_off[c] + before + inc - cnt;
    if (!cnt) return;
    uint32_t* list = a.list[l];
    const unsigned words[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const unsigned w = words[q];
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if ((w >> (8 * b)) & 0xFFu) list[pos++] = off + 4 * q + b;
    }
}

hipError_t launch_compact(const CompactArgs& a, hipStream_t s) {
    const unsigned nchunks = a.chunk_base[a.nlev];
    if (nchunks) hipLaunchKernelGGL(k_count, dim3(nchunks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, a);
    if (nchunks) hipLaunchKernelGGL(k_scatter, dim3(nchunks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace mr
