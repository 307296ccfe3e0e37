// Issue-rate probe of the VALU integer instructions the Montgomery kernels are
// made of (gfx950, wave64).  Each wave runs CH independent chains of one
// instruction; the grid puts W waves on every SIMD (one-wave blocks,
// 4 W blocks per compute unit).  The launch is timed with events; every wave
// also reads the shader cycle counter (clock64, s_memtime) and the
// constant-rate wall counter around its timed loop, which gives the shader
// clock the chip actually ran at under this load.  Lane-operations per cycle
// per compute unit = (lane-operations per second) / (measured clock x CUs).
// Register-only inline assembly: no memory access besides one store per wave.
// v_mad_u64_u32 writes a carry-out SGPR pair that nothing here reads: the
// plain form sends every chain's to VCC, the "own pairs" form gives each chain
// a pair of its own.  AL places each iteration's multiply-adds: 0 where the
// compiler puts them, 1 at addresses 0 modulo 8, 2 at 4 modulo 8 (an
// alignment directive, plus one 4-byte s_nop for 2, ahead of the chains).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <vector>

namespace {

constexpr int kIters = 4096;

template <int OP, int CH, int AL = 0>
__global__ __launch_bounds__(64) void probe(unsigned long long *out, uint32_t seed) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t acc[CH];
    uint64_t cs[CH];  // carry-out pairs (OP 5); nothing reads them
    uint32_t r[CH];
    const uint32_t a = tid * 2654435761u + seed, b = a ^ 0x9e3779b9u;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        acc[c] = tid + c;
        cs[c] = 0;
        r[c] = tid * 7 + c;
    }
    long long t0 = 0, w0 = 0;
    for (int it = -64; it < kIters; ++it) {  // 64 untimed iterations first
        if (it == 0) {
            t0 = clock64();
            w0 = wall_clock64();
        }
        if constexpr (AL == 1) asm volatile(".p2align 3");
        if constexpr (AL == 2) asm volatile(".p2align 3\n\ts_nop 0");
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
            if constexpr (OP == 5)  // the same multiply-add, each chain's carry-out in an SGPR pair of its own
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[c]), "+s"(cs[c]) : "v"(a), "v"(r[c]));
        }
    }
    const long long t1 = clock64(), w1 = wall_clock64();
    uint32_t s = b;
#pragma unroll
    for (int c = 0; c < CH; ++c) s += (uint32_t)acc[c] + (uint32_t)(acc[c] >> 32) + r[c];
    if (threadIdx.x == 0) {
        out[3 * blockIdx.x] = (unsigned long long)(t1 - t0);
        out[3 * blockIdx.x + 1] = (unsigned long long)(w1 - w0);
        out[3 * blockIdx.x + 2] = s;
    }
}

struct Result {
    double clk_mhz;     // shader clock measured by the waves
    double event_rate;  // lane-ops per second from event timing
};

template <int OP, int CH, int AL = 0>
Result run(unsigned long long *d, std::vector<unsigned long long> &h, int waves_per_simd, const hipDeviceProp_t &prop,
           int wall_khz) {
    const int blocks = prop.multiProcessorCount * 4 * waves_per_simd;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hipLaunchKernelGGL((probe<OP, CH, AL>), dim3(blocks), dim3(64), 0, 0, d, 1u);  // warm-up
    (void)hipDeviceSynchronize();
    (void)hipEventRecord(e0);
    hipLaunchKernelGGL((probe<OP, CH, AL>), dim3(blocks), dim3(64), 0, 0, d, 2u);
    (void)hipEventRecord(e1);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipMemcpy(h.data(), d, (size_t)blocks * 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    double clk = 0;
    int n = 0;
    for (int i = 0; i < blocks; ++i)
        if (h[3 * i + 1]) {
            clk += (double)h[3 * i] / (double)h[3 * i + 1];
            ++n;
        }
    const double ops = (double)blocks * 64 * kIters * CH;
    Result res;
    res.clk_mhz = n ? clk / n * wall_khz / 1e3 : 0.0;
    res.event_rate = ops / (ms * 1e-3);
    return res;
}

template <int OP, int CH, int AL = 0>
void report(const char *name, unsigned long long *d, std::vector<unsigned long long> &h, int w,
            const hipDeviceProp_t &prop, int wall_khz) {
    const Result r = run<OP, CH, AL>(d, h, w, prop, wall_khz);
    const double per_cycle = r.clk_mhz > 0 ? r.event_rate / (r.clk_mhz * 1e6) / prop.multiProcessorCount : 0.0;
    std::printf("%-18s waves/SIMD %d chains %2d  %.3e lane-ops/s  clock %5.0f MHz  %6.2f lane-ops/cycle/CU\n", name, w,
                CH, r.event_rate, r.clk_mhz, per_cycle);
}

}  // namespace

int main() {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, 0) != hipSuccess) {
        std::fprintf(stderr, "no HIP device\n");
        return 1;
    }
    int wall_khz = 0;
    if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, 0) != hipSuccess || wall_khz <= 0) {
        std::fprintf(stderr, "no wall clock rate\n");
        return 1;
    }
    std::printf("device %s, %d CUs, peak clock %d kHz, wall counter %d kHz\n", prop.gcnArchName,
                prop.multiProcessorCount, prop.clockRate, wall_khz);
    const int max_blocks = prop.multiProcessorCount * 4 * 8;
    unsigned long long *d = nullptr;
    if (hipMalloc(&d, (size_t)max_blocks * 3 * sizeof(unsigned long long)) != hipSuccess) return 1;
    std::vector<unsigned long long> h((size_t)max_blocks * 3);
    for (int w : {1, 2, 3, 4, 8}) {
        report<0, 1>("v_mad_u64_u32", d, h, w, prop, wall_khz);
        report<0, 2>("v_mad_u64_u32", d, h, w, prop, wall_khz);
        report<0, 4>("v_mad_u64_u32", d, h, w, prop, wall_khz);
        report<0, 8>("v_mad_u64_u32", d, h, w, prop, wall_khz);
        report<0, 16>("v_mad_u64_u32", d, h, w, prop, wall_khz);
    }
    for (int w : {1, 2, 3, 8}) {
        report<5, 16, 1>("own pairs, 0 mod 8", d, h, w, prop, wall_khz);
        report<5, 8, 1>("own pairs, 0 mod 8", d, h, w, prop, wall_khz);
        report<5, 16, 2>("own pairs, 4 mod 8", d, h, w, prop, wall_khz);
        report<5, 8, 2>("own pairs, 4 mod 8", d, h, w, prop, wall_khz);
    }
    for (int w : {1, 2, 3, 4, 8}) {
        report<5, 2>("mad, own pairs", d, h, w, prop, wall_khz);
        report<5, 4>("mad, own pairs", d, h, w, prop, wall_khz);
        report<5, 8>("mad, own pairs", d, h, w, prop, wall_khz);
    }
    for (int w : {1, 4, 8}) {
        report<1, 8>("v_mul_lo_u32", d, h, w, prop, wall_khz);
        report<2, 8>("v_add_co_u32", d, h, w, prop, wall_khz);
        report<3, 8>("v_lshrrev_b64", d, h, w, prop, wall_khz);
        report<4, 8>("v_and_b32", d, h, w, prop, wall_khz);
    }
    (void)hipFree(d);
    return 0;
}
