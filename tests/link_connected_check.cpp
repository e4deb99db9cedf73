// Host driver for the link-connectivity test: reads "n hi lo" lines (an
// upper-link mask over the 2(2^n - 1) rows of Alg. 1, as two hex words) and
// prints 1 if eg::link_connected calls the mask connected, else 0.
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
        switch (n) {
            case 1: c = eg::link_connected<1>((uint64_t)lo); break;
            case 2: c = eg::link_connected<2>((uint64_t)lo); break;
            case 3: c = eg::link_connected<3>((uint64_t)lo); break;
            case 4: c = eg::link_connected<4>((uint64_t)lo); break;
            case 5: c = eg::link_connected<5>((uint64_t)lo); break;
            case 6: c = eg::link_connected<6>(m128); break;
            default: return 2;
        }
        std::printf("%d\n", c ? 1 : 0);
    }
    return 0;
}
