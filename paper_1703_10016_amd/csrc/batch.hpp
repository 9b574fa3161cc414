// Batched persistent assembly: device-side description of a batch and launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "tile_kernel.hpp"

namespace sgbem {

struct BatchConfig {
    int T, S;              // tile edge, strip width
};
constexpr int kNumBatchConfigs = 4;
extern const BatchConfig kBatchConfigs[kNumBatchConfigs];

struct BatchDev {
    CurveDev *curves;      // [n]
    int *npts;             // [n] nodes of each curve (2N)
    int64_t *goff;         // [n] offset of each curve's geometry (in points)
    double *geo;           // [3 * sum npts]: X, Y, J per curve
    TileArgs *args;        // [n]
    TileArgsF *argsf;      // [n]
    int *deg;              // [n] spline degree p
    int *prefix[kNumBatchConfigs];   // [n + 1] first tile of each curve, per tile configuration
};

hipError_t launch_batch_geometry(const BatchDev &d, int n, int max_npts, hipStream_t s);
hipError_t launch_batch_tiles(int cfg, int prec, const BatchDev &d, int n, int total, int grid, hipStream_t s,
                              const KernelEvents *ev = nullptr);
int batch_blocks_per_cu(int cfg, int prec);

}  // namespace sgbem
