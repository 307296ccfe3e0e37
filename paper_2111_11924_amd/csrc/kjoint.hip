// Blinded decryption in one pass per prime (halves_joint_kernel) for every
// size class; the one-lane classes hand the part of a launch that leaves SIMDs
// idle to the lane-group form (kjlanes.hip).  A translation unit of its own,
// so the per-class objects stay as they are.  Its Montgomery products align
// each column (mont.hpp): measured on these kernels' code, that puts their
// multiply-adds at addresses 0 modulo 8.
#define PMK_COLUMN_ALIGN 1
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
    const uint32_t ncu = (uint32_t)device_cus();
    const uint32_t resident = (uint32_t)oj * ncu;
    const uint32_t units = 2 * r.ntiles * lanes_half(CB);
    uint32_t grid = persistent_grid(units, r.slots_dec, r.grid_cap);
    if (grid > resident) grid = resident;
    // the part of a launch that leaves SIMDs idle runs in lane groups, as for
    // the plain CRT halves
    uint32_t main_end = units;
    int L = 1;
    if constexpr (lanes_half(CB) == 1) {
        uint32_t res = resident;
        if (r.grid_cap && r.grid_cap < res) res = r.grid_cap;
        if (r.slots_dec < units && r.slots_dec < res) res = r.slots_dec;  // table room
        uint32_t lane_units = 0;
        L = lanes_for_launch(r, units, res, 4u * ncu, joint_lanes_resident, &lane_units);
        main_end = units - lane_units;
    } else {
        if (wide_fill(r, 2 * r.ntiles, lanes_half(CB), 4u * ncu, joint_lanes_resident(r.cls, 2 * lanes_half(CB)))) {
            L = 2 * lanes_half(CB);
            main_end = 0;
        }
    }
    const uint64_t slot = 2 * table_words_per_slot(r.cls, 1, r.win);  // two odd-power tables
    if (main_end) {
        hipLaunchKernelGGL(halves_joint_kernel<CB>, dim3(persistent_grid(main_end, grid, 0)), dim3(64), 0, s, r, slot,
                           0u, main_end);
        const int e = (int)hipGetLastError();
        if (e) return e;
    }
    if (main_end == units) return 0;
    if (L == 1) {  // the partial round, one lane per number, in a launch of its own
        hipLaunchKernelGGL(halves_joint_kernel<CB>, dim3(persistent_grid(units - main_end, grid, 0)), dim3(64), 0, s,
                           r, slot, main_end, units);
        return (int)hipGetLastError();
    }
    return launch_joint_lanes(r, L, main_end / lanes_half(CB), 2 * r.ntiles, s);
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
