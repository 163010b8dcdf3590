// Prints the wave-neighbour masks of the relaxed synchronisation within a
// diamond tile (pair_neighbours in the kernel header), one line per shape:
// "R DW WX mask_of_wave_0 mask_of_wave_1 ...".  Host code only.
#include <cstdio>
#include "mwd.hpp"

template <int R, int DW>
void dump() {
    using Sh = girih::DiamondShape<R, DW>;
    for (int wx = 1; wx <= 4; ++wx) {
        const int npairs = DW / 2, nwaves = npairs * wx;
        if (nwaves > 16) continue;
        std::printf("%d %d %d", R, DW, wx);
        for (int w = 0; w < nwaves; ++w)
            std::printf(" %u", girih::pair_neighbours<Sh>(w % npairs, npairs, nwaves) & ~(1u << w));
        std::printf("\n");
    }
}

int main() {
    dump<1, 4>();
    dump<1, 8>();
    dump<1, 12>();
    dump<1, 16>();
    dump<1, 24>();
    dump<1, 32>();
    dump<4, 8>();
    dump<4, 16>();
    dump<4, 24>();
    dump<4, 32>();
    return 0;
}
