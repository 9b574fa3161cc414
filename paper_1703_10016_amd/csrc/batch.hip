// Batched assembly of many curves in one persistent launch (fast form,
// n_ref = 1, p in {2, 3, 4}).
//
// The upper-triangle tiles of all matrices form one index space, curve by
// curve (prefix[b] = first tile of curve b).  A persistent grid strides over
// it; each workgroup finds the curve of its tile by binary search in the
// prefix array (the same for every thread of the block), then runs the same
// sweep-and-contract body as the single-matrix kernel with that curve's
// arguments from device memory.  The degree selects one of three compiled
// bodies per tile, so curves of different degree and size share the launch.
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "curve_eval.hpp"
#include "tile_kernel.hpp"

namespace sgbem {

__global__ void batch_geometry_kernel(const CurveDev *curves, const int *npts, const int64_t *goff, double *G)
{
    const int b = blockIdx.y;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int np = npts[b];
    if (n >= np) return;
    double *X = G + 3 * goff[b];
    const double t = double(n) / double(np);
    eval_curve(curves[b], t, X[n], X[np + n], X[2 * np + n]);
}

// Dynamic LDS of the batch kernel: the largest of the tile variants it inlines,
// which share it (static arrays would give each variant its own).
template <typename Real, int T>
constexpr size_t batch_lds_bytes()
{
    const size_t a = TileLds<2, 5, true, Real, T>::bytes(), b = TileLds<2, 7, true, Real, T>::bytes(),
                 c = TileLds<2, 9, true, Real, T>::bytes();
    return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

// FP32: at least 6 waves per SIMD, as for the single-matrix FP32 instances (left
// alone the compiler hoists the sweep's loads into many more registers).
template <typename Real, int T, int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 ? 6 : 1, 8))) void
batch_tile_kernel(const TileArgs *args, const TileArgsF *argsf, const int *deg, const int *prefix, int n, int total)
{
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const int b = lo;
        const TileArgs &a = args[b];
        const TileArgsF &af = argsf[b];
        const int nb = (a.N + T - 1) / T;
        int bi, bj;
        tile_coords(nb, t - prefix[b], bi, bj);
        switch (deg[b]) {   // n_ref = 1: P = 2 nodes per element, Q = 2p + 1 support nodes
        case 2: tile_body<2, 5, 1, true, Real, Real, T, S, true>(a, af, bi, bj); break;
        case 3: tile_body<2, 7, 1, true, Real, Real, T, S, true>(a, af, bi, bj); break;
        default: tile_body<2, 9, 1, true, Real, Real, T, S, true>(a, af, bi, bj); break;
        }
    }
}

hipError_t launch_batch_geometry(const BatchDev &d, int n, int max_npts, hipStream_t s)
{
    dim3 grid((max_npts + 255) / 256, n);
    hipLaunchKernelGGL(batch_geometry_kernel, grid, dim3(256), 0, s, d.curves, d.npts, d.goff, d.geo);
    return hipGetLastError();
}

namespace {
template <typename Real, int T, int S>
hipError_t launch_one(const BatchDev &d, int cfg, int n, int total, int grid, hipStream_t s, const KernelEvents *ev)
{
    constexpr size_t lds = batch_lds_bytes<Real, T>();
    if (ev)
        hipExtLaunchKernelGGL((batch_tile_kernel<Real, T, S>), dim3(grid), dim3(256), lds, s, ev->start, ev->stop, 0,
                              d.args, d.argsf, d.deg, d.prefix[cfg], n, total);
    else
        hipLaunchKernelGGL((batch_tile_kernel<Real, T, S>), dim3(grid), dim3(256), lds, s, d.args, d.argsf, d.deg,
                           d.prefix[cfg], n, total);
    return hipGetLastError();
}
template <typename Real, int T, int S>
int occupancy_one()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_tile_kernel<Real, T, S>, 256, batch_lds_bytes<Real, T>()) !=
        hipSuccess)
        nb = 1;
    return nb < 1 ? 1 : nb;
}
}  // namespace

// 28 x 28 tiles with 7-column strips keep all 256 threads of the sweep busy for
// p = 2..4 (2T + 2p - 1 rows x 4 strips = 236..252 items); the others are the
// tuner's alternatives.
const BatchConfig kBatchConfigs[kNumBatchConfigs] = {{28, 7}, {32, 8}, {24, 6}, {16, 4}};

hipError_t launch_batch_tiles(int cfg, int prec, const BatchDev &d, int n, int total, int grid, hipStream_t s,
                              const KernelEvents *ev)
{
    if (prec == 0) {
        switch (cfg) {
        case 0: return launch_one<double, 28, 7>(d, 0, n, total, grid, s, ev);
        case 1: return launch_one<double, 32, 8>(d, 1, n, total, grid, s, ev);
        case 2: return launch_one<double, 24, 6>(d, 2, n, total, grid, s, ev);
        default: return launch_one<double, 16, 4>(d, 3, n, total, grid, s, ev);
        }
    }
    switch (cfg) {
    case 0: return launch_one<float, 28, 7>(d, 0, n, total, grid, s, ev);
    case 1: return launch_one<float, 32, 8>(d, 1, n, total, grid, s, ev);
    case 2: return launch_one<float, 24, 6>(d, 2, n, total, grid, s, ev);
    default: return launch_one<float, 16, 4>(d, 3, n, total, grid, s, ev);
    }
}

int batch_blocks_per_cu(int cfg, int prec)
{
    if (prec == 0) {
        switch (cfg) {
        case 0: return occupancy_one<double, 28, 7>();
        case 1: return occupancy_one<double, 32, 8>();
        case 2: return occupancy_one<double, 24, 6>();
        default: return occupancy_one<double, 16, 4>();
        }
    }
    switch (cfg) {
    case 0: return occupancy_one<float, 28, 7>();
    case 1: return occupancy_one<float, 32, 8>();
    case 2: return occupancy_one<float, 24, 6>();
    default: return occupancy_one<float, 16, 4>();
    }
}

}  // namespace sgbem
