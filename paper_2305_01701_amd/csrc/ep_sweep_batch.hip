// Batched 2D PT sweep: one persistent launch sweeps the tiles of many
// independent models of different sizes and parameters.
//
// A model table holds one SweepArgs per model (per parity of the ping-pong
// buffers); a tile list holds (model, tile x, tile y) for every tile of the
// models that are still iterating in this precision and tile shape.  The
// grid is sized to the resident capacity of the device and each workgroup
// walks the list with a grid stride; models that converged are simply absent
// from the list, so their tiles cost nothing.  The list length is read from
// device memory, which lets a captured graph of sweeps stay valid while the
// host retires models between replays.
#include "ep_device.h"
#include "ep_tile2d.h"

namespace ep {

namespace {

template <typename R, int TX, int TY, int MODE, int NT = tile_threads_2d<TX, TY>()>
__global__ __launch_bounds__(NT) void k_batch_2d(const SweepArgs<R>* __restrict__ table,
                                                      const TileRef* __restrict__ list,
                                                      const int* __restrict__ count)
{
    const int n = *count;
    // logical workgroup ids contiguous per XCD: consecutive tiles of a model
    // (neighbours, sharing halo lines) run on the same L2
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    for (int t = g; t < n; t += gridDim.x) {
        if (t != g) __syncthreads();        // LDS of the previous tile is still being read
        const TileRef r = list[t];
        sweep_tile_2d<R, TX, TY, MODE, NT>(table[r.model], r.bx, r.by);
    }
}

template <typename R, int TX, int TY, int NT = tile_threads_2d<TX, TY>()>
void run(const SweepArgs<R>* table, const TileRef* list, const int* count, int mode, int grid, hipStream_t s)
{
    if (mode == MODE_CHECK)
        k_batch_2d<R, TX, TY, MODE_CHECK, NT><<<grid, NT, 0, s>>>(table, list, count);
    else if (mode == MODE_PHYS) {
        // physical evaluations run only on single models, with their shape
        if constexpr (TX == 64 && TY == 16)
            k_batch_2d<R, TX, TY, MODE_PHYS, NT><<<grid, NT, 0, s>>>(table, list, count);
    } else
        k_batch_2d<R, TX, TY, MODE_UPDATE, NT><<<grid, NT, 0, s>>>(table, list, count);
}

template <typename R, int TX, int TY, int NT = tile_threads_2d<TX, TY>()>
int occupancy()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_2d<R, TX, TY, MODE_CHECK, NT>, NT, 0) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace

const int kBatchTiles[BATCH_SHAPES][3] = {
    {64, 8, tile_threads_2d<64, 8>()},   {64, 4, tile_threads_2d<64, 4>()},   {32, 8, tile_threads_2d<32, 8>()},
    {128, 4, tile_threads_2d<128, 4>()}, {64, 16, tile_threads_2d<64, 16>()}, {32, 16, tile_threads_2d<32, 16>()}};

template <typename R>
void launch_sweep_batch_2d(int shape, const SweepArgs<R>* table, const TileRef* list, const int* count, int mode,
                           int grid, hipStream_t s)
{
    switch (shape) {
    case 0: run<R, 64, 8>(table, list, count, mode, grid, s); break;
    case 1: run<R, 64, 4>(table, list, count, mode, grid, s); break;
    case 2: run<R, 32, 8>(table, list, count, mode, grid, s); break;
    case 3: run<R, 128, 4>(table, list, count, mode, grid, s); break;
    case 4: run<R, 64, 16>(table, list, count, mode, grid, s); break;
    default: run<R, 32, 16>(table, list, count, mode, grid, s); break;
    }
}

template <typename R>
int batch_blocks_per_cu(int shape)
{
    switch (shape) {
    case 0: return occupancy<R, 64, 8>();
    case 1: return occupancy<R, 64, 4>();
    case 2: return occupancy<R, 32, 8>();
    case 3: return occupancy<R, 128, 4>();
    case 4: return occupancy<R, 64, 16>();
    default: return occupancy<R, 32, 16>();
    }
}

template void launch_sweep_batch_2d<float>(int, const SweepArgs<float>*, const TileRef*, const int*, int, int,
                                           hipStream_t);
template void launch_sweep_batch_2d<double>(int, const SweepArgs<double>*, const TileRef*, const int*, int, int,
                                            hipStream_t);
template int batch_blocks_per_cu<float>(int);
template int batch_blocks_per_cu<double>(int);

}  // namespace ep
