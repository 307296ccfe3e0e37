// Persistent batched encryption for the 4096- and 3072-bit classes: one
// launch whose waves take work units (a quarter tile, 4 lanes per number) from
// a device counter until none is left, then exit -- the parallel loop of
// Algorithm 1's encryption as a work queue.  4096-bit units are numbered
// first, so the last units handed out are the shorter 3072-bit ones.
#include "kernels_impl.hpp"

namespace pmk {

constexpr int kWideLdsEnc =
    lds_words_enc<4096>() > lds_words_enc<3072>() ? lds_words_enc<4096>() : lds_words_enc<3072>();

PMK_DEV uint32_t next_unit(uint32_t *counter) {
    uint32_t u = 0;
    if (threadIdx.x == 0) u = atomicAdd(counter, 1u);
    return __shfl(u, 0, 64);
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void batch_wide_kernel(BatchArgs a) {
    code_align<code_id(kCodeBatchWide, 0, 0)>();
    __shared__ uint32_t lds[kWideLdsEnc];
    uint32_t *tbl = a.table + (size_t)blockIdx.x * a.slot_words;
    const uint32_t total = a.start[kWideClasses];
    for (;;) {
        const uint32_t u = next_unit(a.counter);
        if (u >= total) break;
        if (u < a.start[1])
            encrypt_lanes_unit<4096>(a.runs[0], u, tbl, lds);
        else
            encrypt_lanes_unit<3072>(a.runs[1], u - a.start[1], tbl, lds);
    }
}

// a plain fill kernel (not a memset node), so the reset can sit in a captured graph
__global__ void counter_reset_kernel(uint32_t *counter) {
    if (threadIdx.x == 0) *counter = 0u;
}

int launch_batch(const BatchArgs &a, uint32_t grid, void *stream) {
    hipLaunchKernelGGL(batch_wide_kernel, dim3(grid), dim3(64), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_counter_reset(uint32_t *counter, void *stream) {
    hipLaunchKernelGGL(counter_reset_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, counter);
    return (int)hipGetLastError();
}

uint32_t batch_wave_slots(int num_cus) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)batch_wide_kernel, 64, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return (uint32_t)nb * (uint32_t)num_cus;
}

uint64_t batch_slot_words() {
    uint64_t w = 0;
    for (int i = 0; i < kWideClasses; ++i) {
        const uint64_t x = table_words_per_slot(wide_class(i), 0, 0);
        w = x > w ? x : w;
    }
    return w;
}

}  // namespace pmk
