// hr_reduce.hip -- per-render loss from the wave-tile / tile partials of the
// rasteriser and the path tracer: one wave per render, an FP64 sum of the
// render's partials in index order (lane t takes t, t + 64, ...; then a fixed
// xor tree), times 1 / (pixels * channels).  Single-query and batch kernels
// share the body, so a render's loss is the same bits either way.
#include "hr_kernels.h"

namespace hr {

namespace {

// fixed-order FP64 sum of the tile partials of render r, by one wave
__device__ __forceinline__ void reduce_render(const float* __restrict__ partial, int tiles,
                                              double inv_count, uint64_t r,
                                              double* __restrict__ f) {
  const int lane = threadIdx.x & 63;
  const float* __restrict__ p = partial + r * (uint64_t)tiles;
  double acc = 0.0;
  int t = lane;
  // four loads in flight per lane; the additions keep the order t, t + 64, ...
  for (; t + 192 < tiles; t += 256) {
    const float a = p[t], b = p[t + 64], c = p[t + 128], d = p[t + 192];
    acc += (double)a;
    acc += (double)b;
    acc += (double)c;
    acc += (double)d;
  }
  for (; t < tiles; t += 64) acc += (double)p[t];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) f[r] = acc * inv_count;
}

// one wave per render
__global__ void k_tile_reduce(const float* __restrict__ partial, uint64_t R, int tiles,
                              double inv_count, double* __restrict__ f) {
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t r = blockIdx.x * (uint64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); r < R;
       r += waves)
    reduce_render(partial, tiles, inv_count, r, f);
}

// tile partials -> per-render loss for raster and path-traced queries
__global__ __launch_bounds__(256) void k_batch_reduce(const BatchTable* __restrict__ T) {
  const int nq = T->nq;
  const uint64_t* off = T->off + (uint64_t)kPhReduce * (nq + 1);
  const uint64_t total = off[nq];
  for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = batch_find(off, nq, t);
    const BatchQuery& Q = T->q[q];
    const uint64_t b = (t - off[q]) * (uint64_t)kBatchRenders;
    const uint64_t end = umin64(Q.e.R, b + kBatchRenders);
    for (uint64_t r = b + (threadIdx.x >> 6); r < end; r += (blockDim.x >> 6))
      reduce_render(Q.partial, Q.part_stride, Q.inv_count, r, Q.f);
  }
}

}  // namespace

void launch_tile_reduce(hipStream_t st, const float* partial, uint64_t R, int tiles,
                        double inv_count, double* f) {
  const uint64_t blocks = (R + 3) / 4;
  hipLaunchKernelGGL(k_tile_reduce, dim3((unsigned)umin64(blocks, 1u << 20)), dim3(256), 0, st,
                     partial, R, tiles, inv_count, f);
}

void launch_batch_reduce(hipStream_t st, const BatchTable* T, int blocks) {
  hipLaunchKernelGGL(k_batch_reduce, dim3(blocks), dim3(256), 0, st, T);
}

}  // namespace hr
