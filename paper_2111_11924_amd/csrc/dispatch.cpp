// Dispatch of the per-class launchers (k<bits>.hip) by size-class index.
#include <hip/hip_runtime.h>

#include "pmk_internal.hpp"

namespace pmk {

#define PMK_DECLARE(B)                                                                    \
    int launch_pack_##B(const ClassRun &, const uint8_t *, int, hipStream_t);              \
    int launch_unpack_##B(const ClassRun &, uint8_t *, int, hipStream_t);                  \
    int launch_encrypt_##B(const ClassRun &, hipStream_t);                                 \
    int launch_halves_##B(const ClassRun &, hipStream_t);                                  \
    int launch_garner_##B(const ClassRun &, hipStream_t);                                  \
    uint32_t wave_slots_##B(int, int);                                                     \
    uint64_t slot_words_##B(int, int);
PMK_DECLARE(128)
PMK_DECLARE(256)
PMK_DECLARE(512)
PMK_DECLARE(1024)
PMK_DECLARE(2048)
PMK_DECLARE(3072)
PMK_DECLARE(4096)
PMK_DECLARE(6144)
PMK_DECLARE(8192)

#define PMK_DISPATCH(cls, FN, ...)                          \
    switch (cls) {                                          \
        case 0: return FN##_128(__VA_ARGS__);               \
        case 1: return FN##_256(__VA_ARGS__);               \
        case 2: return FN##_512(__VA_ARGS__);               \
        case 3: return FN##_1024(__VA_ARGS__);              \
        case 4: return FN##_2048(__VA_ARGS__);              \
        case 5: return FN##_3072(__VA_ARGS__);              \
        case 6: return FN##_4096(__VA_ARGS__);              \
        case 7: return FN##_6144(__VA_ARGS__);              \
        case 8: return FN##_8192(__VA_ARGS__);              \
        default: return (int)hipErrorInvalidValue;          \
    }

int launch_pack(const ClassRun &r, const uint8_t *src, int decrypt, void *stream) {
    if (r.ntiles == 0) return 0;
    PMK_DISPATCH(r.cls, launch_pack, r, src, decrypt, (hipStream_t)stream);
}
int launch_unpack(const ClassRun &r, uint8_t *dst, int mode, void *stream) {
    if (r.ntiles == 0) return 0;
    PMK_DISPATCH(r.cls, launch_unpack, r, dst, mode, (hipStream_t)stream);
}
int launch_encrypt(const ClassRun &r, void *stream) {
    if (r.ntiles == 0) return 0;
    PMK_DISPATCH(r.cls, launch_encrypt, r, (hipStream_t)stream);
}
int launch_decrypt_halves(const ClassRun &r, void *stream) {
    if (r.ntiles == 0) return 0;
    PMK_DISPATCH(r.cls, launch_halves, r, (hipStream_t)stream);
}
int launch_garner(const ClassRun &r, void *stream) {
    if (r.ntiles == 0) return 0;
    PMK_DISPATCH(r.cls, launch_garner, r, (hipStream_t)stream);
}
uint64_t table_words_per_slot(int cls, int decrypt, int win) {
    switch (cls) {
        case 0: return slot_words_128(decrypt, win);
        case 1: return slot_words_256(decrypt, win);
        case 2: return slot_words_512(decrypt, win);
        case 3: return slot_words_1024(decrypt, win);
        case 4: return slot_words_2048(decrypt, win);
        case 5: return slot_words_3072(decrypt, win);
        case 6: return slot_words_4096(decrypt, win);
        case 7: return slot_words_6144(decrypt, win);
        case 8: return slot_words_8192(decrypt, win);
        default: return 0;
    }
}

uint32_t exp_units(int cls, int decrypt, uint32_t ntiles) {
    // one wavefront per 64 / L chunks: encryption per tile, CRT halves per tile and prime
    const int bits = kClassBits[cls];
    return decrypt ? 2 * ntiles * (uint32_t)lanes_half(bits) : ntiles * (uint32_t)lanes_full(bits);
}

uint32_t wave_slots(int cls, int decrypt, int num_cus) {
    switch (cls) {
        case 0: return wave_slots_128(decrypt, num_cus);
        case 1: return wave_slots_256(decrypt, num_cus);
        case 2: return wave_slots_512(decrypt, num_cus);
        case 3: return wave_slots_1024(decrypt, num_cus);
        case 4: return wave_slots_2048(decrypt, num_cus);
        case 5: return wave_slots_3072(decrypt, num_cus);
        case 6: return wave_slots_4096(decrypt, num_cus);
        case 7: return wave_slots_6144(decrypt, num_cus);
        case 8: return wave_slots_8192(decrypt, num_cus);
        default: return 1;
    }
}

}  // namespace pmk
