// Exhaustive check of recip_fast (paper_1906_04576_amd/csrc/recip.hpp)
// against the IEEE division 1.0f / d for every float d in [2^-126, 2^126).
// Prints one line "recip_check values <n> mismatches <m>" and exits 0 when
// m == 0.  Built by __graft_entry__.build(); run by the GPU test suite.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "../../paper_1906_04576_amd/csrc/recip.hpp"

__global__ void k_check(unsigned long long* mismatches, unsigned* first, unsigned lo, unsigned hi) {
    const unsigned base = lo + (blockIdx.x * 256u + threadIdx.x) * 64u;
    unsigned long long c = 0;
    for (unsigned j = 0; j < 64; ++j) {
        const unsigned i = base + j;
        if (i >= hi) break;
        const float d = __builtin_bit_cast(float, i);
        if (__builtin_bit_cast(unsigned, 1.0f / d) != __builtin_bit_cast(unsigned, mr::recip_fast(d))) {
            ++c;
            atomicMin(first, i);
        }
    }
    if (c) atomicAdd(mismatches, c);
}

int main() {
    const unsigned lo = 0x00800000u, hi = 0x7E800000u;  // 2^-126 .. 2^126 (exclusive)
    unsigned long long* mism = nullptr;
    unsigned* first = nullptr;
    if (hipMalloc(&mism, sizeof(unsigned long long)) != hipSuccess || hipMalloc(&first, sizeof(unsigned)) != hipSuccess) {
        printf("recip_check: allocation failed\n");
        return 2;
    }
    const unsigned long long zero = 0;
    const unsigned none = 0xFFFFFFFFu;
    if (hipMemcpy(mism, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(first, &none, sizeof(none), hipMemcpyHostToDevice) != hipSuccess) {
        printf("recip_check: copy failed\n");
        return 2;
    }
    const unsigned n = hi - lo, threads = (n + 63) / 64, blocks = (threads + 255) / 256;
    hipLaunchKernelGGL(k_check, dim3(blocks), dim3(256), 0, 0, mism, first, lo, hi);
    unsigned long long m = 0;
    unsigned f = 0;
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(&m, mism, sizeof(m), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&f, first, sizeof(f), hipMemcpyDeviceToHost) != hipSuccess) {
        printf("recip_check: kernel failed\n");
        return 2;
    }
    printf("recip_check values %u mismatches %llu first 0x%08x\n", n, m, m ? f : 0u);
    hipFree(mism);
    hipFree(first);
    return m == 0 ? 0 : 1;
}
