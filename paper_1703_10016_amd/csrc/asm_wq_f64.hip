// Instantiations of the tile kernel for weighted-quadrature row assembly in FP64: one kernel per
// (degree p, points per element P); written by gen_instances.py.
#include "tile_kernel.hpp"

namespace sgbem {

hipError_t launch_wq_f64(int p, int P, const TileArgs &a, hipStream_t s, const KernelEvents *ev)
{
    switch (p * 16 + P) {
    case 18: return a.N >= 4096 ? launch_tile<2, 3, 1, true, double, 28, 7, 4>(a, s, ev) : launch_tile<2, 3, 1, true, double, 28, 7>(a, s, ev);
    case 20: return launch_tile<4, 7, 1, true, double, 28, 7>(a, s, ev);
    case 22: return launch_tile<6, 11, 1, true, double, 20, 5>(a, s, ev);
    case 24: return launch_tile<8, 15, 1, true, double, 28, 7>(a, s, ev);
    case 34: return a.N >= 4096 ? launch_tile<2, 5, 1, true, double, 28, 7, 4>(a, s, ev) : launch_tile<2, 5, 1, true, double, 28, 7>(a, s, ev);
    case 36: return launch_tile<4, 11, 1, true, double, 28, 7>(a, s, ev);
    case 38: return launch_tile<6, 17, 1, true, double, 16, 8>(a, s, ev);
    case 40: return launch_tile<8, 23, 1, true, double, 16, 8>(a, s, ev);
    case 50: return a.N >= 4096 ? launch_tile<2, 7, 1, true, double, 28, 7, 4>(a, s, ev) : launch_tile<2, 7, 1, true, double, 28, 7>(a, s, ev);
    case 52: return launch_tile<4, 15, 1, true, double, 28, 7>(a, s, ev);
    case 54: return launch_tile<6, 23, 1, true, double, 16, 8>(a, s, ev);
    case 56: return launch_tile<8, 31, 1, true, double, 16, 8>(a, s, ev);
    case 66: return a.N >= 4096 ? launch_tile<2, 9, 1, true, double, 28, 7, 4>(a, s, ev) : launch_tile<2, 9, 1, true, double, 28, 7>(a, s, ev);
    case 68: return launch_tile<4, 19, 1, true, double, 28, 7>(a, s, ev);
    case 70: return launch_tile<6, 29, 1, true, double, 16, 8>(a, s, ev);
    case 72: return launch_tile<8, 39, 1, true, double, 16, 8>(a, s, ev);
    case 82: return launch_tile<2, 11, 1, true, double, 24, 6>(a, s, ev);
    case 84: return launch_tile<4, 23, 1, true, double, 24, 6>(a, s, ev);
    case 86: return launch_tile<6, 35, 1, true, double, 32, 8>(a, s, ev);
    case 88: return launch_tile<8, 47, 1, true, double, 32, 8>(a, s, ev);
    case 98: return launch_tile<2, 13, 1, true, double, 24, 6>(a, s, ev);
    case 100: return launch_tile<4, 27, 1, true, double, 32, 8>(a, s, ev);
    case 102: return launch_tile<6, 41, 1, true, double, 32, 8>(a, s, ev);
    case 104: return launch_tile<8, 55, 1, true, double, 32, 8>(a, s, ev);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sgbem
