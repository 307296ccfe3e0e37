// Persistent batched exponentiation for the multi-lane classes (4096 and
// 3072 bits): one launch whose waves take work units (tiles, or CRT jobs of a
// tile) from a device counter until none is left, then exit -- the parallel
// loops of Algorithm 1 as a work queue.  4096-bit units are numbered first, so
// the last units handed out are the shorter 3072-bit ones.
#include "kernels_impl.hpp"

namespace pmk {

constexpr int kWideLdsDec = lds_words_dec<4096>() > lds_words_dec<3072>() ? lds_words_dec<4096>() : lds_words_dec<3072>();
constexpr int kWideLdsEnc =
    lds_words_enc<4096>() > lds_words_enc<3072>() ? lds_words_enc<4096>() : lds_words_enc<3072>();

PMK_DEV uint32_t next_unit(uint32_t *counter) {
    uint32_t u = 0;
    if (threadIdx.x == 0) u = atomicAdd(counter, 1u);
    return __shfl(u, 0, 64);
}

template <bool DEC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void batch_wide_kernel(BatchArgs a) {
    __shared__ uint32_t lds[DEC ? kWideLdsDec : kWideLdsEnc];
    uint32_t *tbl = a.table + (size_t)blockIdx.x * a.slot_words;
    const uint32_t total = a.start[kWideClasses];
    for (;;) {
        const uint32_t u = next_unit(a.counter);
        if (u >= total) break;
        if (u < a.start[1]) {
            if constexpr (DEC) halves_lanes_unit<4096>(a.runs[0], u, tbl, lds);
            else encrypt_lanes_unit<4096>(a.runs[0], u, tbl, lds);
        } else {
            if constexpr (DEC) halves_lanes_unit<3072>(a.runs[1], u - a.start[1], tbl, lds);
            else encrypt_lanes_unit<3072>(a.runs[1], u - a.start[1], tbl, lds);
        }
    }
}

// a plain fill kernel (not a memset node), so the reset can sit in a captured graph
__global__ void counter_reset_kernel(uint32_t *counter) {
    if (threadIdx.x == 0) *counter = 0u;
}

int launch_batch(const BatchArgs &a, int decrypt, uint32_t grid, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (decrypt)
        hipLaunchKernelGGL(batch_wide_kernel<true>, dim3(grid), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL(batch_wide_kernel<false>, dim3(grid), dim3(64), 0, s, a);
    return (int)hipGetLastError();
}

int launch_counter_reset(uint32_t *counter, void *stream) {
    hipLaunchKernelGGL(counter_reset_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, counter);
    return (int)hipGetLastError();
}

uint32_t batch_wave_slots(int decrypt, int num_cus) {
    int nb = 0;
    const void *fn = decrypt ? (const void *)batch_wide_kernel<true> : (const void *)batch_wide_kernel<false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64, 0) != hipSuccess || nb < 1) nb = 1;
    return (uint32_t)nb * (uint32_t)num_cus;
}

uint64_t batch_slot_words(int decrypt, const int *win) {
    uint64_t w = 0;
    for (int i = 0; i < kWideClasses; ++i) {
        const uint64_t x = table_words_per_slot(wide_class(i), decrypt, win[i]);
        w = x > w ? x : w;
    }
    return w;
}

}  // namespace pmk
