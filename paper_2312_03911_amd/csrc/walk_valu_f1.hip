// Instantiations of the vector-ALU walk for float runs with 1 coordinate(s) per
// lane (one translation unit per set, so the build compiles them in parallel).
#include "walk_valu.h"

namespace ggns {

hipError_t launch_walk_valu_f1(void *arena, const RunDev *runs, const Tile *tiles, int n_tiles, int var, int gf,
                          size_t lds, int phase, hipStream_t s) {
    return launch_walk_t<float, 1>(arena, runs, tiles, n_tiles, var, gf, lds, phase, s);
}

}  // namespace ggns
