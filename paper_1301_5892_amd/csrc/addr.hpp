#pragma once
// A 64-bit device address carried through 32-bit lane intrinsics
// (readfirstlane works on int): split into its low and high words and joined
// back, each word widened through unsigned, never sign-extended.  A low word
// with bit 31 set is an ordinary address; widening it through a signed int
// would set the whole high word.  Usable from host code (tested there) and
// device code.
#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIP__)
#define VOG_HD __host__ __device__
#else
#define VOG_HD
#endif

namespace vog {

VOG_HD inline constexpr int addr_lo(uint64_t a) { return (int)(uint32_t)a; }
VOG_HD inline constexpr int addr_hi(uint64_t a) { return (int)(uint32_t)(a >> 32); }
VOG_HD inline constexpr uint64_t addr_join(int lo, int hi) {
    return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

}  // namespace vog
