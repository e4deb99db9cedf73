// Host driver for the link-connectivity test: reads "n hi lo" lines (a
// non-empty upper-link mask over the 2(2^n - 1) rows of Alg. 1, as two hex
// words) and prints whether eg::link_connected calls it connected (1 or 0)
// and eg::link_component of it (the component of its lowest row, two hex
// words).
#include <hip/hip_runtime.h>

#include <cstdio>

#include "eg_link.h"

int main()
{
    int n;
    unsigned long long hi, lo;
    while (std::scanf("%d %llx %llx", &n, &hi, &lo) == 3) {
        const unsigned __int128 m128 = ((unsigned __int128)hi << 64) | lo;
        bool c = false;
        unsigned __int128 comp = 0;
        switch (n) {
            case 1: c = eg::link_connected<1>((uint64_t)lo), comp = eg::link_component<1>((uint64_t)lo); break;
            case 2: c = eg::link_connected<2>((uint64_t)lo), comp = eg::link_component<2>((uint64_t)lo); break;
            case 3: c = eg::link_connected<3>((uint64_t)lo), comp = eg::link_component<3>((uint64_t)lo); break;
            case 4: c = eg::link_connected<4>((uint64_t)lo), comp = eg::link_component<4>((uint64_t)lo); break;
            case 5: c = eg::link_connected<5>((uint64_t)lo), comp = eg::link_component<5>((uint64_t)lo); break;
            case 6: c = eg::link_connected<6>(m128), comp = eg::link_component<6>(m128); break;
            default: return 2;
        }
        std::printf("%d %llx %llx\n", c ? 1 : 0, (unsigned long long)(comp >> 64), (unsigned long long)comp);
    }
    return 0;
}
