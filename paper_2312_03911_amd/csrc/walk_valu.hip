// Launch of the vector-ALU walk: the class's precision and coordinates per
// lane pick the instantiation (each compiled in its own translation unit).
#include "ggns_common.h"

namespace ggns {

#define GGNS_WALK_VALU_DECL(NAME)                                                                  \
    hipError_t NAME(void *arena, const RunDev *runs, const Tile *tiles, int n_tiles, int var, int gf, \
                    size_t lds, int phase, hipStream_t s);
GGNS_WALK_VALU_DECL(launch_walk_valu_d1)
GGNS_WALK_VALU_DECL(launch_walk_valu_d2)
GGNS_WALK_VALU_DECL(launch_walk_valu_d4)
GGNS_WALK_VALU_DECL(launch_walk_valu_f1)
GGNS_WALK_VALU_DECL(launch_walk_valu_f2)
GGNS_WALK_VALU_DECL(launch_walk_valu_f4)
GGNS_WALK_VALU_DECL(launch_walk_valu_f8)
#undef GGNS_WALK_VALU_DECL

int launch_walk_class(void *arena, const RunDev *runs_dev, const Tile *tiles, int n_tiles, int prec,
                      int C, int var, int gf, size_t lds, int phase, hipStream_t s) {
    hipError_t e = hipErrorInvalidValue;
    if (prec == GGNS_FP64) {
        switch (C) {
            case 1: e = launch_walk_valu_d1(arena, runs_dev, tiles, n_tiles, var, gf, lds, phase, s); break;
            case 2: e = launch_walk_valu_d2(arena, runs_dev, tiles, n_tiles, var, gf, lds, phase, s); break;
            case 4: e = launch_walk_valu_d4(arena, runs_dev, tiles, n_tiles, var, gf, lds, phase, s); break;
        }
    } else {
        switch (C) {
            case 1: e = launch_walk_valu_f1(arena, runs_dev, tiles, n_tiles, var, gf, lds, phase, s); break;
            case 2: e = launch_walk_valu_f2(arena, runs_dev, tiles, n_tiles, var, gf, lds, phase, s); break;
            case 4: e = launch_walk_valu_f4(arena, runs_dev, tiles, n_tiles, var, gf, lds, phase, s); break;
            case 8: e = launch_walk_valu_f8(arena, runs_dev, tiles, n_tiles, var, gf, lds, phase, s); break;
        }
    }
    return e == hipSuccess ? GGNS_OK : GGNS_EHIP;
}

}  // namespace ggns
