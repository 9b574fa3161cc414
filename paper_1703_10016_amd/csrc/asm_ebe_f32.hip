// Instantiations of the tile kernel for the element-by-element far part in FP32: one kernel per
// (degree p, points per element P); written by gen_instances.py.
#include "tile_kernel.hpp"

namespace sgbem {

hipError_t launch_ebe_f32(int p, int P, const TileArgs &a, hipStream_t s, const KernelEvents *ev)
{
    switch (p * 16 + P) {
    case 17: return launch_tile<1, 2, 0, false, float, 32, 8>(a, s, ev);
    case 18: return launch_tile<2, 4, 0, false, float, 28, 7>(a, s, ev);
    case 19: return launch_tile<3, 6, 0, false, float, 20, 5>(a, s, ev);
    case 20: return launch_tile<4, 8, 0, false, float, 28, 7>(a, s, ev);
    case 21: return launch_tile<5, 10, 0, false, float, 24, 6>(a, s, ev);
    case 22: return launch_tile<6, 12, 0, false, float, 20, 5>(a, s, ev);
    case 23: return launch_tile<7, 14, 0, false, float, 32, 8>(a, s, ev);
    case 24: return launch_tile<8, 16, 0, false, float, 28, 7>(a, s, ev);
    case 33: return launch_tile<1, 3, 0, false, float, 32, 8>(a, s, ev);
    case 34: return launch_tile<2, 6, 0, false, float, 28, 7>(a, s, ev);
    case 35: return launch_tile<3, 9, 0, false, float, 24, 8>(a, s, ev);
    case 36: return launch_tile<4, 12, 0, false, float, 28, 7>(a, s, ev);
    case 37: return launch_tile<5, 15, 0, false, float, 32, 8>(a, s, ev);
    case 38: return launch_tile<6, 18, 0, false, float, 28, 7>(a, s, ev);
    case 39: return launch_tile<7, 21, 0, false, float, 32, 8>(a, s, ev);
    case 40: return launch_tile<8, 24, 0, false, float, 28, 7>(a, s, ev);
    case 49: return launch_tile<1, 4, 0, false, float, 32, 8>(a, s, ev);
    case 50: return launch_tile<2, 8, 0, false, float, 28, 7>(a, s, ev);
    case 51: return launch_tile<3, 12, 0, false, float, 24, 8>(a, s, ev);
    case 52: return launch_tile<4, 16, 0, false, float, 28, 7>(a, s, ev);
    case 53: return launch_tile<5, 20, 0, false, float, 32, 8>(a, s, ev);
    case 54: return launch_tile<6, 24, 0, false, float, 24, 8>(a, s, ev);
    case 55: return launch_tile<7, 28, 0, false, float, 32, 8>(a, s, ev);
    case 56: return launch_tile<8, 32, 0, false, float, 28, 7>(a, s, ev);
    case 65: return launch_tile<1, 5, 0, false, float, 32, 8>(a, s, ev);
    case 66: return launch_tile<2, 10, 0, false, float, 28, 7>(a, s, ev);
    case 67: return launch_tile<3, 15, 0, false, float, 24, 8>(a, s, ev);
    case 68: return launch_tile<4, 20, 0, false, float, 28, 7>(a, s, ev);
    case 69: return launch_tile<5, 25, 0, false, float, 32, 8>(a, s, ev);
    case 70: return launch_tile<6, 30, 0, false, float, 24, 8>(a, s, ev);
    case 71: return launch_tile<7, 35, 0, false, float, 32, 8>(a, s, ev);
    case 72: return launch_tile<8, 40, 0, false, float, 28, 7>(a, s, ev);
    case 81: return launch_tile<1, 6, 0, false, float, 32, 8>(a, s, ev);
    case 82: return launch_tile<2, 12, 0, false, float, 24, 6>(a, s, ev);
    case 83: return launch_tile<3, 18, 0, false, float, 32, 8>(a, s, ev);
    case 84: return launch_tile<4, 24, 0, false, float, 32, 8>(a, s, ev);
    case 85: return launch_tile<5, 30, 0, false, float, 32, 8>(a, s, ev);
    case 86: return launch_tile<6, 36, 0, false, float, 32, 8>(a, s, ev);
    case 87: return launch_tile<7, 42, 0, false, float, 28, 7>(a, s, ev);
    case 88: return launch_tile<8, 48, 0, false, float, 32, 8>(a, s, ev);
    case 97: return launch_tile<1, 7, 0, false, float, 32, 8>(a, s, ev);
    case 98: return launch_tile<2, 14, 0, false, float, 24, 6>(a, s, ev);
    case 99: return launch_tile<3, 21, 0, false, float, 32, 8>(a, s, ev);
    case 100: return launch_tile<4, 28, 0, false, float, 32, 8>(a, s, ev);
    case 101: return launch_tile<5, 35, 0, false, float, 32, 8>(a, s, ev);
    case 102: return launch_tile<6, 42, 0, false, float, 32, 8>(a, s, ev);
    case 103: return launch_tile<7, 49, 0, false, float, 28, 7>(a, s, ev);
    case 104: return launch_tile<8, 56, 0, false, float, 32, 8>(a, s, ev);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sgbem
