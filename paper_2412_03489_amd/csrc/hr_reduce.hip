// hr_reduce.hip -- per-render loss from the wave-tile / tile partials of the
// rasteriser and the path tracer (layout part_index: groups of 16 renders,
// tile-major).  One wave per group of 16 renders: lane (q, i) = (lane / 16,
// lane % 16) sums, in FP64 and in tile order, the partials of render i of the
// group over the tiles t = q, q + 4, q + 8, ...; the four runs are then added
// in the order q = 0, 1, 2, 3, times 1 / (pixels * channels).  Single-query
// and batch kernels share the body, so a render's loss is the same bits
// either way.
#include "hr_kernels.h"

namespace hr {

namespace {

// fixed-order FP64 sums of the tile partials of renders [16 g, 16 g + 16)
// (those below R), by one wave
__device__ __forceinline__ void reduce_group(const float* __restrict__ partial, int tiles,
                                             double inv_count, uint64_t g, uint64_t R,
                                             double* __restrict__ f) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, q = lane >> 4;
  const float* __restrict__ p = partial + g * (uint64_t)tiles * 16u + i;
  double acc = 0.0;
  int t = q;
  // four loads in flight per lane; the additions keep the order t, t + 4, ...
  for (; t + 12 < tiles; t += 16) {
    const float a = p[t * 16], b = p[(t + 4) * 16], c = p[(t + 8) * 16], d = p[(t + 12) * 16];
    acc += (double)a;
    acc += (double)b;
    acc += (double)c;
    acc += (double)d;
  }
  for (; t < tiles; t += 4) acc += (double)p[t * 16];
  const double a1 = __shfl(acc, i + 16, 64);
  const double a2 = __shfl(acc, i + 32, 64);
  const double a3 = __shfl(acc, i + 48, 64);
  const uint64_t r = g * 16u + (uint64_t)i;
  if (q == 0 && r < R) f[r] = (((acc + a1) + a2) + a3) * inv_count;
}

// one wave per group of 16 renders
__global__ void k_tile_reduce(const float* __restrict__ partial, uint64_t R, int tiles,
                              double inv_count, double* __restrict__ f, const int* skip) {
  if (skip && *skip) return;
  const uint64_t groups = (R + 15) / 16;
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t g = blockIdx.x * (uint64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); g < groups;
       g += waves)
    reduce_group(partial, tiles, inv_count, g, R, f);
}

// tile partials -> per-render loss for raster and path-traced queries; a task
// is a run of kBatchRenders renders (a multiple of 16), one wave per group
__global__ __launch_bounds__(256) void k_batch_reduce(const BatchTable* __restrict__ T) {
  static_assert(kBatchRenders % 16 == 0, "reduce tasks hold whole groups of 16 renders");
  const int nq = T->nq;
  const uint64_t* off = T->off + (uint64_t)kPhReduce * (nq + 1);
  const uint64_t total = off[nq];
  for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = batch_find(off, nq, t);
    const BatchQuery& Q = T->q[q];
    const uint64_t b = (t - off[q]) * (uint64_t)kBatchRenders;
    const uint64_t end = umin64(Q.e.L, b + kBatchRenders);
    for (uint64_t g = b / 16 + (threadIdx.x >> 6); g * 16 < end; g += (blockDim.x >> 6))
      reduce_group(Q.partial, Q.part_stride, Q.inv_count, g, Q.e.L, Q.f);
  }
}

}  // namespace

void launch_tile_reduce(hipStream_t st, const float* partial, uint64_t R, int tiles,
                        double inv_count, double* f, const int* skip) {
  const uint64_t blocks = ((R + 15) / 16 + 3) / 4;
  hipLaunchKernelGGL(k_tile_reduce, dim3((unsigned)umin64(blocks, 1u << 20)), dim3(256), 0, st,
                     partial, R, tiles, inv_count, f, skip);
}

void launch_batch_reduce(hipStream_t st, const BatchTable* T, int blocks) {
  hipLaunchKernelGGL(k_batch_reduce, dim3(blocks), dim3(256), 0, st, T);
}

}  // namespace hr
