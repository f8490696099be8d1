// Reference Philox4x32-10 bijection taken from rocRAND's engine (a library
// routine, used only to pin the oracle's independent implementation).
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) and prints the four output words.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct Exposed : rocrand_device::philox4x32_10_engine {
    uint4 bijection(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    Exposed e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.bijection(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
