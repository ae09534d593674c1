// Test helper: prints Philox4x32-10 blocks computed by rocRAND's open-source
// engine on the host, as an implementation independent of the oracle's.
// Input lines on stdin: c0 c1 c2 c3 k0 k1 (hex); output: r0 r1 r2 r3 (hex).
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Exposed : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    Exposed eng;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = eng.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
