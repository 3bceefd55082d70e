// Host check of the address split/join the kernels use to move a 64-bit
// base address through 32-bit lane intrinsics (addr.hpp).  Prints one line
// per case: "ok" or "bad <address>".
#include <stdint.h>
#include <stdio.h>

#include "addr.hpp"

// The same split followed by the sign-extending join the kernels must avoid.
static uint64_t join_sign_extended(int lo, int hi) {
    return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(int64_t)lo;
}

int main() {
    const uint64_t cases[] = {0x0000000000000000ull, 0x00007f1200000000ull, 0x00007f127fffff00ull,
                              0x00007f1280000000ull, 0x00007f12fffffff0ull, 0x00007fffffffff00ull,
                              0x0000100080000100ull, 0xffffffff80000000ull};
    int bad = 0, differs = 0;
    for (uint64_t a : cases) {
        const uint64_t b = vog::addr_join(vog::addr_lo(a), vog::addr_hi(a));
        if (b != a) {
            printf("bad %016llx\n", (unsigned long long)a);
            ++bad;
        }
        if (join_sign_extended(vog::addr_lo(a), vog::addr_hi(a)) != a) ++differs;
    }
    // the sign-extending join must get every low word with bit 31 set wrong
    // (here 4 of the cases) whenever the high word is not all ones
    printf("%s %d\n", bad ? "FAIL" : "ok", differs);
    return bad ? 1 : 0;
}
