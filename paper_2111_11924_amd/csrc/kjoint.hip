// Blinded decryption in one pass per prime (halves_joint_kernel) for every
// size class.  A translation unit of its own, so the per-class objects stay as
// they are.
#include "kernels_impl.hpp"

namespace pmk {

namespace {

template <int CB>
int launch_joint_class(const ClassRun &r, hipStream_t s) {
    // resident blocks on this device; never more than the r.slots_dec table slots
    // (those of the CRT-halves kernel, which is at least as occupied and capped by
    // the same unit count)
    static const int oj = [] {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)halves_joint_kernel<CB>, 64, 0) !=
                hipSuccess ||
            nb < 1)
            nb = 1;
        return nb;
    }();
    int dev = 0, ncu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        ncu = 1;
    const uint64_t resident = (uint64_t)oj * (uint64_t)ncu;
    const uint32_t units = 2 * r.ntiles * lanes_half(CB);
    uint64_t grid = persistent_grid(units, r.slots_dec, r.grid_cap);
    if (grid > resident) grid = resident;
    const uint64_t slot = 2 * table_words_per_slot(r.cls, 1, r.win);  // two odd-power tables
    hipLaunchKernelGGL(halves_joint_kernel<CB>, dim3((uint32_t)grid), dim3(64), 0, s, r, slot);
    return (int)hipGetLastError();
}

}  // namespace

int launch_decrypt_joint(const ClassRun &r, void *stream) {
    if (r.ntiles == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    switch (r.cls) {
        case 0: return launch_joint_class<128>(r, s);
        case 1: return launch_joint_class<256>(r, s);
        case 2: return launch_joint_class<512>(r, s);
        case 3: return launch_joint_class<1024>(r, s);
        case 4: return launch_joint_class<2048>(r, s);
        case 5: return launch_joint_class<3072>(r, s);
        case 6: return launch_joint_class<4096>(r, s);
        case 7: return launch_joint_class<6144>(r, s);
        case 8: return launch_joint_class<8192>(r, s);
        default: return (int)hipErrorNotSupported;
    }
}

}  // namespace pmk
