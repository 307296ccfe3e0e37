// Issue-rate probe of the VALU integer instructions the Montgomery kernels are
// made of (gfx950, wave64): each thread runs CH independent chains of one
// instruction, the grid fills every compute unit, and the rate is reported in
// lane-operations per clock per compute unit (64 = one per lane per clock).
// The v_mad_u64_u32 figure is the measured ceiling the CRT kernels are
// compared against beside the nominal one-per-lane-per-clock peak.
// Register-only inline assembly: no memory access besides one store per thread.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int kIters = 2048;

template <int OP, int CH>
__global__ __launch_bounds__(256) void probe(uint32_t *out, uint32_t seed) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t acc[CH];
    uint32_t r[CH];
    const uint32_t a = tid * 2654435761u + seed, b = a ^ 0x9e3779b9u;
    for (int c = 0; c < CH; ++c) {
        acc[c] = tid + c;
        r[c] = tid * 7 + c;
    }
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if constexpr (OP == 0)  // 32x32 -> 64 multiply with 64-bit accumulate
                asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(acc[c]) : "v"(a), "v"(r[c]) : "vcc");
            if constexpr (OP == 1)
                asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(r[c]) : "v"(a));
            if constexpr (OP == 2)
                asm volatile("v_add_co_u32 %0, vcc, %0, %1" : "+v"(r[c]) : "v"(a) : "vcc");
            if constexpr (OP == 3)
                asm volatile("v_lshrrev_b64 %0, 28, %0" : "+v"(acc[c]));
            if constexpr (OP == 4)
                asm volatile("v_and_b32 %0, 0xfffffff, %0" : "+v"(r[c]));
        }
    }
    uint32_t s = b;
    for (int c = 0; c < CH; ++c) s += (uint32_t)acc[c] + (uint32_t)(acc[c] >> 32) + r[c];
    out[tid] = s;
}

template <int OP, int CH>
float time_ms(uint32_t *d, int blocks) {
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hipLaunchKernelGGL((probe<OP, CH>), dim3(blocks), dim3(256), 0, 0, d, 1u);
    (void)hipDeviceSynchronize();
    (void)hipEventRecord(e0);
    for (int i = 0; i < 3; ++i) hipLaunchKernelGGL((probe<OP, CH>), dim3(blocks), dim3(256), 0, 0, d, (uint32_t)i);
    (void)hipEventRecord(e1);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / 3;
}

template <int OP, int CH>
void report(const char *name, uint32_t *d, int blocks, const hipDeviceProp_t &prop) {
    const float ms = time_ms<OP, CH>(d, blocks);
    const double ops = (double)blocks * 256 * kIters * CH;
    const double rate = ops / (ms * 1e-3);
    const double clk = prop.clockRate * 1e3;
    std::printf("%-16s chains %2d  %8.3f ms  %.3e lane-ops/s  %6.2f lane-ops/clk/CU\n", name, CH, ms, rate,
                rate / clk / prop.multiProcessorCount);
}

}  // namespace

int main() {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, 0) != hipSuccess) {
        std::fprintf(stderr, "no HIP device\n");
        return 1;
    }
    std::printf("device %s, %d CUs, clock %d kHz\n", prop.gcnArchName, prop.multiProcessorCount, prop.clockRate);
    const int blocks = prop.multiProcessorCount * 8;  // 8 blocks of 4 waves per CU: 8 waves per SIMD
    uint32_t *d = nullptr;
    if (hipMalloc(&d, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) return 1;
    report<0, 4>("v_mad_u64_u32", d, blocks, prop);
    report<0, 8>("v_mad_u64_u32", d, blocks, prop);
    report<0, 16>("v_mad_u64_u32", d, blocks, prop);
    report<1, 8>("v_mul_lo_u32", d, blocks, prop);
    report<2, 8>("v_add_co_u32", d, blocks, prop);
    report<3, 8>("v_lshrrev_b64", d, blocks, prop);
    report<4, 8>("v_and_b32", d, blocks, prop);
    (void)hipFree(d);
    return 0;
}
