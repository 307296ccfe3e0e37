// Blinded decryption (one pass per prime, Sec. 3.1) in lane groups
// (halves_lanes_joint_kernel) for the part of a launch that leaves SIMDs idle:
// the one-lane classes (128- to 4096-bit keys) with 2 or 4 lanes per number as
// lanes_for_launch decides, the lane-group classes (6144/8192) with 8 instead
// of 4 as wide_fill decides.  A translation unit of its own, so the other
// objects stay as they are and the classes compile in parallel with them.
#include "kernels_impl.hpp"

namespace pmk {

namespace {

template <int CB, int L>
uint32_t resident_of() {
    static const uint32_t nb = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)halves_lanes_joint_kernel<CB, L>, 64, 0) !=
                hipSuccess ||
            n < 1)
            n = 1;
        return (uint32_t)n;
    }();
    return nb * (uint32_t)device_cus();
}

template <int CB, int L>
int launch_class(const ClassRun &r, uint32_t jt_begin, uint32_t jt_end, hipStream_t s) {
    constexpr Geom G = make_geom(CB);
    constexpr uint64_t K = lane_limbs(G, L) / L;
    // two odd-power tables (T1 for c*, T2 for c_R), each lane's K limbs
    const uint64_t slot = 2 * (uint64_t)(1u << (r.win - 1)) * K * kTile;
    const uint32_t units = (jt_end - jt_begin) * L;
    // L / lanes_half lane-group slots fit one slot of the class's own blinded
    // kernel (2 tables of at least 2^(win-1) entries of nla >= K L limbs)
    uint32_t grid = persistent_grid(units, r.slots_dec * (uint32_t)(L / lanes_half(CB)), r.grid_cap);
    grid = std::min(grid, resident_of<CB, L>());
    hipLaunchKernelGGL((halves_lanes_joint_kernel<CB, L>), dim3(grid), dim3(64), 0, s, r, slot, jt_begin * L,
                       jt_end * L);
    return (int)hipGetLastError();
}

template <int CB>
int launch_L(const ClassRun &r, int L, uint32_t jt_begin, uint32_t jt_end, hipStream_t s) {
    if constexpr (lanes_half(CB) == 1) {
        if (L == 2) return launch_class<CB, 2>(r, jt_begin, jt_end, s);
        if (L == 4) return launch_class<CB, 4>(r, jt_begin, jt_end, s);
        if constexpr (eight_lanes(CB))
            if (L == 8) return launch_class<CB, 8>(r, jt_begin, jt_end, s);
    } else {
        if (L == 2 * lanes_half(CB)) return launch_class<CB, 2 * lanes_half(CB)>(r, jt_begin, jt_end, s);
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace

uint32_t joint_lanes_resident(int cls, int L) {
    switch (cls * 16 + L) {
        case 0 * 16 + 2: return resident_of<128, 2>();
        case 0 * 16 + 4: return resident_of<128, 4>();
        case 1 * 16 + 2: return resident_of<256, 2>();
        case 1 * 16 + 4: return resident_of<256, 4>();
        case 2 * 16 + 2: return resident_of<512, 2>();
        case 2 * 16 + 4: return resident_of<512, 4>();
        case 3 * 16 + 2: return resident_of<1024, 2>();
        case 3 * 16 + 4: return resident_of<1024, 4>();
        case 4 * 16 + 2: return resident_of<2048, 2>();
        case 4 * 16 + 4: return resident_of<2048, 4>();
        case 4 * 16 + 8: return resident_of<2048, 8>();
        case 5 * 16 + 2: return resident_of<3072, 2>();
        case 5 * 16 + 4: return resident_of<3072, 4>();
        case 5 * 16 + 8: return resident_of<3072, 8>();
        case 6 * 16 + 2: return resident_of<4096, 2>();
        case 6 * 16 + 4: return resident_of<4096, 4>();
        case 6 * 16 + 8: return resident_of<4096, 8>();
        case 7 * 16 + 2 * lanes_half(6144): return resident_of<6144, 2 * lanes_half(6144)>();
        case 8 * 16 + 2 * lanes_half(8192): return resident_of<8192, 2 * lanes_half(8192)>();
        default: return 0;
    }
}

int launch_joint_lanes(const ClassRun &r, int L, uint32_t jt_begin, uint32_t jt_end, void *stream) {
    if (jt_end <= jt_begin) return 0;
    hipStream_t s = (hipStream_t)stream;
    switch (r.cls) {
        case 0: return launch_L<128>(r, L, jt_begin, jt_end, s);
        case 1: return launch_L<256>(r, L, jt_begin, jt_end, s);
        case 2: return launch_L<512>(r, L, jt_begin, jt_end, s);
        case 3: return launch_L<1024>(r, L, jt_begin, jt_end, s);
        case 4: return launch_L<2048>(r, L, jt_begin, jt_end, s);
        case 5: return launch_L<3072>(r, L, jt_begin, jt_end, s);
        case 6: return launch_L<4096>(r, L, jt_begin, jt_end, s);
        case 7: return launch_L<6144>(r, L, jt_begin, jt_end, s);
        case 8: return launch_L<8192>(r, L, jt_begin, jt_end, s);
        default: return (int)hipErrorNotSupported;
    }
}

}  // namespace pmk
