// hr_raster.hip -- perturbed disk records and the fused rasterise + MSE kernel.
//
// One render = the disk scene at theta_r = theta (+- h u) - a tau_s.  The
// loss of a render is the mean over H*W*C of (I - T)^2 (the image loss of the
// paper's tasks, section "Methods").  Work decomposition:
//   block (256 threads = 4 wave64) = four 16x16 wave tiles (arranged 2x2,
//   4x1 or 1x4) x S consecutive renders; each lane owns one pixel column of 4
//   rows of its wave tile, and the target tile lives in registers for all S
//   renders.  Per pass a wave loads disk records (one disk per lane; up to 32
//   disks lanes 0-31 and 32-63 hold two renders, so one cull serves both; the
//   next pass's records already in flight), culls them against its wave tile
//   with a conservative circle/rectangle test, and walks each render's
//   surviving disks in painter's order as a wave-uniform bit mask; with at
//   most 64 disks the lanes park the records next to the disks' colours in
//   LDS and a survivor's record is one broadcast LDS read, otherwise it comes
//   by lane broadcasts.  Per pixel only the LDS address of the top disk's
//   colour is kept.
//
// Coverage is decided exactly as the FP64 definition: every record carries
// r^2 widened and narrowed by the FP32 error band of the test; the FP32 test
// against the narrowed r^2 is exact outside the band, and a disk with any
// pixel inside its band takes a wave-uniform branch that rebuilds that disk's
// unrounded parameters and decides those pixels in FP64 (rare).
//
// A wave tile that no disk reaches renders as background; its loss is the
// tile's sum of T^2, computed once per block with the same arithmetic.  Per
// render each wave folds its lanes in quads (two DPP adds) and parks the 16
// quad sums in LDS; every 16 renders the wave sums each render's 16 in a
// fixed order, giving one FP32 partial per (render, wave tile) -- the same
// bits for any block shape and any S.
#include <type_traits>

#include "hr_device.h"
#include "hr_kernels.h"

namespace hr {

namespace {

typedef const RasterExact __attribute__((address_space(4))) ConstExact;
constexpr int kSub = 16;         // wave tile side (pixels)
constexpr int kRows = 4;         // rows per lane
constexpr int kMaxS = 256;       // renders per block (upper bound)
constexpr int kFlush = 16;       // renders whose quad partials a wave holds in LDS
// the flush reads the wave's kFlush x 16 quad partials as one float4 per lane
static_assert(kFlush * 16 == 64 * 4, "a flush covers exactly one float4 per lane");
constexpr float kFar = 1.0e18f;  // centre of pixels outside the image

// record: (cx, cy, (r^2 + band)(1 + 1e-5), r^2 - band) in FP32; r <= 0: never covered
__device__ __forceinline__ void record_one(const double* __restrict__ theta,
                                           const double* __restrict__ tau,
                                           const double* __restrict__ u,
                                           const float* __restrict__ radius, int n, int D, int ppd,
                                           int A, int NH, double h, uint64_t gid,
                                           float4* __restrict__ rec) {
  // render r = (draw * A + a) * NH + shift with A, NH in {1, 2}: one division
  // (32-bit while the index fits) and bit operations
  int k;
  uint64_t r;
  if (gid >> 32 == 0) {
    const uint32_t r32 = (uint32_t)gid / (uint32_t)D;
    k = (int)((uint32_t)gid - r32 * (uint32_t)D);
    r = r32;
  } else {
    r = gid / (uint64_t)D;
    k = (int)(gid - r * (uint64_t)D);
  }
  const int sh = NH == 2 ? (int)(r & 1u) : 0;
  const uint64_t rem = NH == 2 ? r >> 1 : r;
  const int ai = A == 2 ? (int)(rem & 1u) : 0;
  const uint64_t sidx = A == 2 ? rem >> 1 : rem;
  const double* t = tau + sidx * (uint64_t)n;
  const double a = ai == 0 ? 1.0 : -1.0;
  const double shift = sh == 0 ? h : -h;
  double p[3];
  for (int q = 0; q < ppd; ++q) {
    const int j = k * ppd + q;
    double base = theta[j];
    if (NH == 2) base = base + shift * u[j];
    p[q] = base - a * t[j];
  }
  const double rad = ppd == 3 ? p[2] : (double)radius[k];
  float4 out = make_float4((float)p[0], (float)p[1], -1.0f, -1.0f);
  if (rad > 0.0) {
    // r^2 +- band; the upper value is also the cull radius, widened by a
    // further 1e-5 relative so that culling stays conservative in FP32
    const double r2 = (double)(float)(rad * rad);
    const double band = ambiguity_band(p[0], p[1], rad);
    out.z = (float)((r2 + band) * 1.00001);
    out.w = (float)(r2 - band);
  }
  rec[gid] = out;
}

__global__ void k_records(const double* __restrict__ theta, const double* __restrict__ tau,
                          const double* __restrict__ u, const float* __restrict__ radius,
                          int n, int D, int ppd, int A, int NH, double h, uint64_t total,
                          float4* __restrict__ rec, const int* skip) {
  if (skip && *skip) return;
  for (uint64_t gid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; gid < total;
       gid += (uint64_t)gridDim.x * blockDim.x)
    record_one(theta, tau, u, radius, n, D, ppd, A, NH, h, gid, rec);
}

// Exact coverage of pixel (x, y) by disk k of render r, in FP64 from the
// unrounded parameters theta (+- h u) - a tau (the definition the FP32 test
// approximates).
__device__ __noinline__ bool cover_fp64(RasterExact ex, uint64_t r, int k, int x, int y, int W,
                                        int H) {
  const int sh = (int)(r % (uint64_t)ex.NH);
  const uint64_t rem = r / (uint64_t)ex.NH;
  const int ai = (int)(rem % (uint64_t)ex.A);
  const uint64_t sidx = rem / (uint64_t)ex.A;
  const double a = ai == 0 ? 1.0 : -1.0;
  const double shift = sh == 0 ? ex.h : -ex.h;
  double p[3];
  for (int q = 0; q < ex.ppd; ++q) {
    const int j = k * ex.ppd + q;
    double base = ex.theta[j];
    if (ex.tau) {
      if (ex.NH == 2) base = base + shift * ex.u[j];
      base = base - a * ex.tau[sidx * (uint64_t)ex.n + j];
    }
    p[q] = base;
  }
  const double rad = ex.ppd == 3 ? p[2] : (double)ex.radius[k];
  const double px = ((double)x + 0.5) / (double)W, py = ((double)y + 0.5) / (double)H;
  const double dx = px - p[0], dy = py - p[1];
  return rad > 0.0 && dx * dx + dy * dy < rad * rad;
}

__device__ __forceinline__ float dpp_quad_sum(float v) {
  // lanes (0,1,2,3) of every quad end with the quad's sum: xor 1, then xor 2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));
  return v;
}

__device__ __forceinline__ float lane_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// float4 slots of the colour table (see raster_block)
__host__ __device__ inline int raster_table_slots(int D) {
  return D <= 32 ? 8 * (D + 1) * 2 : (D <= 64 ? 4 * (D + 1) * 2 : D + 1);
}

// Coverage of the wave's pixels by one surviving disk s = (cx, cy, r^2 + band,
// r^2 - band) with colour address id: per row the pixel's top-disk address
// becomes id where the FP32 test decides (d^2 < r^2 - band); pixels inside the
// band are decided in FP64 from the unrounded parameters (rare, wave-uniform
// branch).
__device__ __forceinline__ void cover_disk(const float4 s, int k, uint32_t id,
                                           float px, const float (&py)[kRows],
                                           uint32_t (&idx)[kRows], const ConstExact* exq, uint64_t r,
                                           int x, int yb, int W, int H, int lane) {
  const float dx = px - s.x;
  const float dx2 = dx * dx;
  uint64_t amb[kRows];   // lanes whose squared distance fell inside the band
  uint64_t amb_any = 0;
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const float dy = py[i] - s.y;
    const float d2 = fmaf(dy, dy, dx2);
    // lane masks straight from the compares (v_cmp into SGPRs)
    const uint64_t m_hi = __builtin_amdgcn_fcmpf(d2, s.z, 4 /* ordered < */);
    const uint64_t m_lo = __builtin_amdgcn_fcmpf(d2, s.w, 4 /* ordered < */);
    amb[i] = m_hi & ~m_lo;
    amb_any |= amb[i];
    idx[i] = d2 < s.w ? id : idx[i];
  }
  if (amb_any) {
    // the parameters of this rare path are read here, through an address the
    // compiler cannot see through, so that they do not hold scalar registers
    // for the whole render loop
    uint64_t ex_addr = (uint64_t)exq;
    __asm__ volatile("" : "+s"(ex_addr));
    const ConstExact& ex = *(const ConstExact*)ex_addr;
    const int sh = (int)(r % (uint64_t)ex.NH);
    const uint64_t rem = r / (uint64_t)ex.NH;
    const double a = (rem % (uint64_t)ex.A) == 0 ? 1.0 : -1.0;
    const double* ts = ex.tau + (rem / (uint64_t)ex.A) * (uint64_t)ex.n;
    const double shift = sh == 0 ? ex.h : -ex.h;
    double p[3];
    for (int qq = 0; qq < ex.ppd; ++qq) {
      const int jj = k * ex.ppd + qq;
      double base = ex.theta[jj];
      if (ex.NH == 2) base = base + shift * ex.u[jj];
      p[qq] = base - a * ts[jj];
    }
    const double rad = ex.ppd == 3 ? p[2] : (double)ex.radius[k];
    const double dxd = ((double)x + 0.5) / (double)W - p[0];
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      if ((amb[i] >> lane) & 1) {
        const double dyd = ((double)(yb + i) + 0.5) / (double)H - p[1];
        const bool cov = rad > 0.0 && dxd * dxd + dyd * dyd < rad * rad;
        idx[i] = cov ? id : idx[i];
      }
    }
  }
}

typedef float lds_f4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) lds_f4 LdsF4;

// Loss of one render on the wave's tile, given the lane mask of the disks that
// survived the cull (bit l = disk l): a survivor's record is one broadcast LDS
// read at its entry's address in the wave's table col0 (entry 0 =
// background, stride 32 B: record, then colour), the address its covered
// pixels keep.  Returns the lane-quad sum of the pixels' squared errors (every
// lane of a quad holds it).
template <int C>
__device__ __forceinline__ float render_survivors(
    uint64_t mask, float px, const float (&py)[kRows], const float (&tm2)[kRows][C], float t2,
    float e_empty, uint32_t col0, const float* s_cc, const ConstExact* ex, uint64_t r, int x, int yb,
    int W, int H, int lane) {
  if (mask == 0) return e_empty;
  uint32_t idx[kRows];
#pragma unroll
  for (int i = 0; i < kRows; ++i) idx[i] = col0;
  while (mask) {
    const int l = __builtin_ctzll(mask);
    mask &= mask - 1;
    const uint32_t id = col0 + (uint32_t)(l + 1) * 32u;
    const lds_f4 v = *(const LdsF4*)(uintptr_t)id;
    cover_disk(make_float4(v.x, v.y, v.z, v.w), l, id, px, py, idx, ex, r, x, yb, W, H, lane);
  }
  float e = t2;
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const lds_f4 col = *(const LdsF4*)(uintptr_t)(idx[i] + (uint32_t)sizeof(float4));
    const float cc[4] = {col.x, col.y, col.z, col.w};
    float pe = C == 4 ? s_cc[(idx[i] - col0) / 32u] : col.w;
#pragma unroll
    for (int c = 0; c < C; ++c) pe = fmaf(cc[c], tm2[i][c], pe);
    e += pe;
  }
  return dpp_quad_sum(e);
}

// Cull of the records q the lanes hold against the wave tile (centre mx, my,
// half extent hx, hy), after parking each in its table slot (LDS byte address
// rec_slot) for the survivors' broadcast reads.  The [0, 1] clamp (an output
// modifier) can only shorten the distance, so no covering disk is dropped;
// r <= 0 records carry r^2 = -1 and never pass; lanes outside dmask (repeats
// of the last disk, or a render past the end) are masked out.
__device__ __forceinline__ uint64_t park_and_cull(const float4 q, uint32_t rec_slot,
                                                  uint64_t dmask, float mx, float my, float hx,
                                                  float hy) {
  *(LdsF4*)(uintptr_t)rec_slot = lds_f4{q.x, q.y, q.z, q.w};
  const float ddx = __builtin_amdgcn_fmed3f(fabsf(q.x - mx) - hx, 0.0f, 1.0f);
  const float ddy = __builtin_amdgcn_fmed3f(fabsf(q.y - my) - hy, 0.0f, 1.0f);
  return __builtin_amdgcn_fcmpf(fmaf(ddy, ddy, ddx * ddx), q.z, 5 /* ordered <= */) & dmask;
}

// One block's work: renders [r0, r0 + nr) of one query on one block of four
// 16x16 wave tiles (2x2, 4x1 or 1x4).
// Shared by the per-query kernel and the persistent batch kernel, so a render's
// tile partial is the same bits whichever launch computes it.
template <int C, bool kOneGroup, class Query>
__device__ __forceinline__ void raster_block(const Query& a, const ConstExact* exq, int tile,
                                             uint64_t r0, int nr, float4* smem) {
  const int W = a.W, H = a.H, D = a.D, tiles_x = a.tiles_x, bwx = a.bwx;
  const int subs_x = a.subs_x;
  const uint64_t subs = (uint64_t)a.subs;
  const float4* __restrict__ rec = a.rec;
  const float* __restrict__ target = a.target;
  const float* __restrict__ colors = a.colors;
  float* __restrict__ partial = a.partial;
  const ConstExact* ex = exq;
  const uint64_t r_base = a.r_base;
  // colour table, entry 0 = background.  Up to 64 disks every wave has its
  // own table (two up to 32 disks, one per render of a cull pass) whose entry
  // k + 1 holds disk k's record of the render in flight followed by disk k's
  // colour (stride 32 B; a pixel keeps the entry's address); beyond 64 disks
  // the block shares one table of colours (stride 16 B; a pixel keeps the
  // colour's address).
  float4* s_col = smem;
  const int tab_slots = raster_table_slots(D);
  float* s_q = (float*)(smem + tab_slots);     // [4 waves][kFlush][16] quad partials
  float* s_cc = s_q + 4 * kFlush * 16;         // D + 1 squared norms (C == 4)
  __syncthreads();   // the previous work item's readers of LDS are done

  // channels, and |c|^2 in .w (C <= 3) or in s_cc (C == 4)
  const int ntab = kOneGroup ? (D <= 32 ? 8 : 4) : 1;   // tables of the block
  for (int t = threadIdx.x; t < ntab * (D + 1); t += blockDim.x) {
    const int k = t % (D + 1);
    float cc[4] = {0.f, 0.f, 0.f, 0.f};
    if (k > 0)
      for (int c = 0; c < C; ++c) cc[c] = colors[(size_t)(k - 1) * C + c];
    float n2 = 0.0f;
    for (int c = 0; c < C; ++c) n2 = fmaf(cc[c], cc[c], n2);
    s_col[kOneGroup ? 2 * t + 1 : t] = make_float4(cc[0], cc[1], cc[2], C == 4 ? cc[3] : n2);
    if (C == 4 && t <= D) s_cc[k] = n2;
  }

  // the wave index is wave-uniform: said so, everything derived from it
  // (tile origin, liveness, the render loop bound) stays in scalar registers
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int bx0 = (tile % tiles_x) * (kSub * bwx), by0 = (tile / tiles_x) * (kSub * a.bwy);
  const int tx0 = bx0 + (wave % bwx) * kSub;
  const int ty0 = by0 + (wave / bwx) * kSub;
  // a wave tile wholly outside the image renders nothing and writes no partial
  const bool live = tx0 < W && ty0 < H;
  const int x = tx0 + (lane & 15);
  const int yb = ty0 + (lane >> 4) * kRows;
  const float invW = 1.0f / (float)W, invH = 1.0f / (float)H;
  const float px = x < W ? ((float)x + 0.5f) / (float)W : kFar;
  // per pixel loss written as |T|^2 + (|c|^2 - 2 c.T): the lane keeps -2T
  // in registers and the sum of |T|^2 over its pixels; a background pixel
  // (c = 0) adds exactly nothing to the second part
  float py[kRows];
  float tm2[kRows][C];
  float t2 = 0.0f;
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int y = yb + i;
    const bool valid = (x < W) && (y < H);
    py[i] = y < H ? ((float)y + 0.5f) / (float)H : kFar;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float t = valid ? target[((size_t)y * W + x) * C + c] : 0.0f;
      tm2[i][c] = -2.0f * t;
      t2 = fmaf(t, t, t2);
    }
  }
  // loss of an all-background sub-tile: the same arithmetic as the main path
  const float e_empty = dpp_quad_sum(t2);
  // sub-tile rectangle of pixel centres (centre, half extent), widened by a
  // slack far above FP32 rounding so that culling never drops a covering disk
  const float mx = ((float)tx0 + 0.5f * kSub) * invW, hx = (0.5f * kSub - 0.5f) * invW + 4e-6f;
  const float my = ((float)ty0 + 0.5f * kSub) * invH, hy = (0.5f * kSub - 0.5f) * invH + 4e-6f;
  __syncthreads();

  const float4* rp0 = rec + r0 * (uint64_t)D;
  const int nr_wave = live ? nr : 0;
  // per pixel state: the LDS byte address of the top disk's colour; the
  // colour table opens the dynamic LDS, which starts after the static LDS
  const uint32_t col0 = __builtin_amdgcn_groupstaticsize();
  // the wave's quad partials of up to kFlush renders, [render][quad]; the
  // quad heads write them, and every kFlush renders the wave sums each
  // render's 16 in a fixed order into the wave tile's loss partial
  float* s_qw = s_q + wave * kFlush * 16;
  float* sq = s_qw + (lane >> 2);
  const bool quad_head = (lane & 3) == 0;
  const uint64_t sub_w = (uint64_t)(ty0 / kSub) * (uint64_t)subs_x + (uint64_t)(tx0 / kSub);
  // renders [f0, f0 + cnt) of the block: lane 4j + i adds quads 4i..4i+3 of
  // render f0 + j, the lane quad adds the four sums (two DPP adds)
  auto flush = [&](int f0, int cnt) {
    typedef float lds_f4v __attribute__((ext_vector_type(4)));
    const lds_f4v v = *(const __attribute__((address_space(3))) lds_f4v*)(uintptr_t)(
        s_qw + lane * 4);
    const float acc = dpp_quad_sum(((v.x + v.y) + v.z) + v.w);
    const int j = lane >> 2;
    if (quad_head && j < cnt)
      partial[part_index(r_base + r0 + (uint64_t)(f0 + j), sub_w, subs)] = acc;
  };
  if constexpr (kOneGroup) {
    // Up to 32 disks, lanes 0-31 hold the records of one render and lanes
    // 32-63 those of the next, so one cull serves two renders, each half with
    // its own table; up to 64 disks, lane l holds disk l of one render.  The
    // next pass's records are loaded while this one is processed, alternating
    // between two register sets.
    auto passes = [&](auto g) {
      constexpr int G = decltype(g)::value;   // renders per cull
      const int half = G == 2 ? lane >> 5 : 0;
      const int lane_d = min(G == 2 ? lane & 31 : lane, D - 1);
      const uint64_t dm = D < 64 ? (1ull << D) - 1 : ~0ull;
      const char* rb = (const char*)rp0;
      const uint64_t rstride = (uint64_t)D * sizeof(float4);
      const uint32_t loff = (uint32_t)half * (uint32_t)rstride + (uint32_t)lane_d * 16u;
      // this wave's G tables and this lane's record slot in them
      const uint32_t colw = col0 + (uint32_t)(wave * G * (D + 1)) * 32u;
      const uint32_t colb = colw + (uint32_t)(D + 1) * 32u;
      const uint32_t rec_slot = colw + (uint32_t)(half * (D + 1) + lane_d + 1) * 32u;
      // the block's records as one buffer of nr * D records, the lane's byte
      // offset in a vector register and the pass's in a scalar one (no
      // address arithmetic on the vector unit; descriptor word 3 is the gfx9
      // raw buffer format, 32-bit data); lanes past the buffer's end read
      // zeros
      typedef float g_f4 __attribute__((ext_vector_type(4)));
      const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
          (void*)rb, (short)0, (int)((uint64_t)nr * rstride), 0x00020000);
      auto lane_rec = [&](int rr) {
        const uint32_t r1 = (uint32_t)min(rr, nr - 1);
        const g_f4 v = __builtin_bit_cast(
            g_f4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)loff,
                                                         (int)(r1 * (uint32_t)rstride), 0));
        return make_float4(v.x, v.y, v.z, v.w);
      };
      // lanes that take part in the cull of the pass starting at render rr
      auto pass_mask = [&](int rr) {
        return G == 2 ? (rr + 1 < nr_wave ? dm | (dm << 32) : dm) : dm;
      };
      const uint64_t rq = r_base + r0;
      float4 qa = lane_rec(0);
      // kFlush is a multiple of 2 * G: a flush group ends after whole passes
      for (int f0 = 0; f0 < nr_wave; f0 += kFlush) {
        const int fe = min(f0 + kFlush, nr_wave);
        float* sqr = sq;   // advanced by two passes' partials
        for (int rr = f0; rr < fe; rr += 2 * G) {
          const float4 qb = lane_rec(rr + G);
          uint64_t m = park_and_cull(qa, rec_slot, pass_mask(rr), mx, my, hx, hy);
          float e = render_survivors<C>(m & dm, px, py, tm2, t2, e_empty, colw, s_cc, ex,
                                        rq + (uint64_t)rr, x, yb, W, H, lane);
          if (quad_head) sqr[0] = e;
          if (G == 2 && rr + 1 < nr_wave) {
            e = render_survivors<C>(m >> 32, px, py, tm2, t2, e_empty, colb, s_cc, ex,
                                    rq + (uint64_t)(rr + 1), x, yb, W, H, lane);
            if (quad_head) sqr[16] = e;
          }
          if (rr + G >= nr_wave) break;
          qa = lane_rec(rr + 2 * G);
          m = park_and_cull(qb, rec_slot, pass_mask(rr + G), mx, my, hx, hy);
          e = render_survivors<C>(m & dm, px, py, tm2, t2, e_empty, colw, s_cc, ex,
                                  rq + (uint64_t)(rr + G), x, yb, W, H, lane);
          if (quad_head) sqr[G * 16] = e;
          if (G == 2 && rr + 3 < nr_wave) {
            e = render_survivors<C>(m >> 32, px, py, tm2, t2, e_empty, colb, s_cc, ex,
                                    rq + (uint64_t)(rr + 3), x, yb, W, H, lane);
            if (quad_head) sqr[48] = e;
          }
          sqr += 2 * G * 16;
        }
        flush(f0, fe - f0);
      }
    };
    if (D <= 32)
      passes(std::integral_constant<int, 2>{});
    else
      passes(std::integral_constant<int, 1>{});
  } else {
    for (int rr = 0; rr < nr_wave; ++rr) {
      const float4* rp = rp0 + (uint64_t)rr * D;
      const uint64_t r = r_base + r0 + (uint64_t)rr;
      uint32_t idx[kRows];
#pragma unroll
      for (int i = 0; i < kRows; ++i) idx[i] = col0;
      uint64_t any = 0;
      for (int g0 = 0; g0 < D; g0 += 64) {
        const int k = g0 + lane;
        const float4 q = k < D ? rp[k] : make_float4(0.f, 0.f, -1.f, -1.f);
        const float ddx = fmaxf(fabsf(q.x - mx) - hx, 0.0f);
        const float ddy = fmaxf(fabsf(q.y - my) - hy, 0.0f);
        uint64_t mask = __builtin_amdgcn_fcmpf(fmaf(ddy, ddy, ddx * ddx), q.z, 5 /* <= */);
        any |= mask;
        while (mask) {
          const int l = __builtin_ctzll(mask);
          mask &= mask - 1;
          const float4 sd = make_float4(lane_bcast(q.x, l), lane_bcast(q.y, l),
                                        lane_bcast(q.z, l), lane_bcast(q.w, l));
          cover_disk(sd, g0 + l, col0 + (uint32_t)(g0 + l + 1) * (uint32_t)sizeof(float4), px, py,
                     idx, ex, r, x, yb, W, H, lane);
        }
      }
      float e;
      if (any == 0) {
        e = e_empty;
      } else {
        e = t2;
#pragma unroll
        for (int i = 0; i < kRows; ++i) {
          typedef float lds_f4 __attribute__((ext_vector_type(4)));
          const lds_f4 col = *(const __attribute__((address_space(3))) lds_f4*)(uintptr_t)idx[i];
          const float cc[4] = {col.x, col.y, col.z, col.w};
          float pe = C == 4 ? s_cc[(idx[i] - col0) / (uint32_t)sizeof(float4)] : col.w;
#pragma unroll
          for (int c = 0; c < C; ++c) pe = fmaf(cc[c], tm2[i][c], pe);
          e += pe;
        }
        e = dpp_quad_sum(e);
      }
      if (quad_head) sq[(rr % kFlush) * 16] = e;
      if ((rr + 1) % kFlush == 0 || rr + 1 == nr_wave) flush(rr - rr % kFlush, rr % kFlush + 1);
    }
  }
}

// At least 7 waves per SIMD: caps the kernel at 72 VGPRs.  Left to itself the
// scheduler spends more registers on loads in flight in the loss fold and the
// occupancy drops to 5-6 waves, which costs more than those loads gain.
template <int C, bool kOneGroup>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7)))
void k_raster_loss(RasterQuery a, uint64_t chunks) {
  extern __shared__ float4 smem[];
  if (a.skip && *a.skip) return;
  // XCD-aware order: consecutive blocks on one XCD (block id mod 8) sweep all
  // tiles of one render chunk, so a chunk's records stay in that XCD's L2.
  const uint64_t b = blockIdx.x;
  const uint64_t xcd = b & 7u, j = b >> 3;
  const uint64_t chunk = (j / (uint64_t)a.tiles) * 8u + xcd;
  const int tile = (int)(j % (uint64_t)a.tiles);
  if (chunk >= chunks) return;
  const uint64_t r0 = chunk * (uint64_t)a.S;
  const int nr = (int)min((uint64_t)a.S, a.R - r0);
  // the query's exact-path parameters where they sit in the kernel arguments
  // (the query is the first argument)
  const ConstExact* exq = (const ConstExact*)((const __attribute__((address_space(4))) char*)
                                                  __builtin_amdgcn_kernarg_segment_ptr() +
                                              offsetof(RasterQuery, ex));
  raster_block<C, kOneGroup, RasterQuery>(a, exq, tile, r0, nr, smem);
}

// single render at theta, coverage in FP64 (the definition)
__global__ void k_render_disks(RasterExact ex, const float* __restrict__ colors, int W, int H,
                               int C, int D, float* __restrict__ image) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W || y >= H) return;
  int top = -1;
  for (int k = 0; k < D; ++k)
    if (cover_fp64(ex, 0, k, x, y, W, H)) top = k;
  for (int c = 0; c < C; ++c)
    image[((size_t)y * W + x) * C + c] = top >= 0 ? colors[(size_t)top * C + c] : 0.0f;
}

// ---- batch kernels ----
typedef const RasterQuery __attribute__((address_space(4))) ConstRasterQuery;
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__global__ __launch_bounds__(256) void k_batch_records(const BatchTable* __restrict__ T) {
  const int nq = T->nq;
  const uint64_t* off = T->off + (uint64_t)kPhRecords * (nq + 1);
  const uint64_t total = off[nq];
  for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = batch_find(off, nq, t);
    const BatchQuery& Q = T->q[q];
    const EstShape& e = Q.e;
    const uint64_t b = (t - off[q]) * (uint64_t)kBatchElems;
    const uint64_t end = umin64(e.R * (uint64_t)Q.ds.D, b + kBatchElems);
    for (uint64_t g = b + threadIdx.x; g < end; g += blockDim.x)
      record_one(Q.theta, Q.tau, Q.u, Q.ds.radius, e.n, Q.ds.D, Q.ds.ppd, e.A, e.NH, e.h, g,
                 Q.rec);
  }
}

// Persistent raster over the eight work queues of one raster class (channel
// count C, all disks in one wavefront or not).  Queue x holds the chunks of
// S renders whose position in the class's chunk sequence is x mod 8, each
// chunk as one item per block of its image; blocks start on the queue of
// their XCD (block id mod 8), so the records of a chunk are read by one XCD,
// and move on to the other queues when theirs is empty.  Every item is
// claimed by exactly one atomic increment; a block leaves after seeing all
// eight queues exhausted.
// At least 7 waves per SIMD, as k_raster_loss.
template <int C, bool kOneGroup>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7)))
void k_batch_raster(const BatchTable* __restrict__ T) {
  extern __shared__ float4 smem[];
  __shared__ unsigned long long s_item;
  const WorkQueues& W = T->raster[raster_class(C, kOneGroup ? 1 : 65)];
  const int home = blockIdx.x & 7;
  uint64_t all = 0;
  for (int x = 0; x < 8; ++x) all += W.items[x];
  if (all == 0) return;   // nothing of this kind in the batch
  for (int k = 0; k < 8; ++k) {
    const int x = (home + k) & 7;
    const uint64_t nitems = W.items[x];
    const uint64_t sb = W.seg_off[x], se = W.seg_off[x + 1];
    if (threadIdx.x == 0) s_item = atomicAdd(&W.ctr[x], 1ull);
    __syncthreads();
    uint64_t it = uniform64(s_item);
    __syncthreads();   // every thread has read s_item before it is reused
    while (it < nitems) {
      // claim the next item now: the counter's round trip overlaps this
      // item's work (the claimed item is this block's next, whatever it is)
      unsigned long long next = 0;
      if (threadIdx.x == 0) next = atomicAdd(&W.ctr[x], 1ull);
      // segment of the item: largest s in [sb, se) with seg[s].item0 <= it
      uint64_t lo = sb, hi = se - 1;
      while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (uniform64(W.seg[mid].item0) <= it) lo = mid; else hi = mid - 1;
      }
      const WorkSeg sg = uniform_copy(&W.seg[lo]);
      // the query descriptor is read through the constant address space: the
      // batch never writes it, so its fields come in by scalar loads on use
      const ConstRasterQuery& a = *(const ConstRasterQuery*)(&T->q[sg.q].rq);
      const uint64_t l = it - sg.item0;
      const uint64_t chunk = (uint64_t)sg.c0 + 8u * (l / (uint64_t)sg.tiles);
      const int tile = (int)(l % (uint64_t)sg.tiles);
      const uint64_t r0 = chunk * (uint64_t)a.S;
      const int nr = (int)min((uint64_t)a.S, a.R - r0);
      raster_block<C, kOneGroup, ConstRasterQuery>(a, &a.ex, tile, r0, nr, smem);
      if (threadIdx.x == 0) s_item = next;
      __syncthreads();
      it = uniform64(s_item);
      __syncthreads();
    }
  }
}

inline unsigned grid_for(uint64_t total, int block) {
  uint64_t g = (total + block - 1) / block;
  return (unsigned)(g > 65536u * 16u ? 65536u * 16u : (g == 0 ? 1 : g));
}

}  // namespace

void launch_records(hipStream_t st, const EstShape& e, const DiskScene& s, const double* theta,
                    const double* tau, const double* u, float4* rec) {
  const uint64_t total = e.R * (uint64_t)s.D;
  hipLaunchKernelGGL(k_records, dim3(grid_for(total, 256)), dim3(256), 0, st, theta, tau, u,
                     s.radius, e.n, s.D, s.ppd, e.A, e.NH, e.h, total, rec, e.skip);
}

int raster_subtiles(int W, int H) { return ((W + kSub - 1) / kSub) * ((H + kSub - 1) / kSub); }

// shape 0 (the library's choice): of the three block shapes, the one that
// covers the W x H image with the fewest blocks; ties go to the 16x64 column of
// four wave tiles, then to 32x32.  A 256x256 image needs 64 blocks of each
// shape, and there the column is 3% faster than 32x32 and 16% faster than
// 64x16; an image only two wave tiles wide or tall would leave half of a
// column's (or a row's) wave tiles idle
void raster_block_shape(int shape, int W, int H, int* bwx, int* bwy) {
  if (shape <= 0 || shape > 3) {
    const int64_t sx = (W + kSub - 1) / kSub, sy = (H + kSub - 1) / kSub;
    auto blocks = [&](int64_t bx) { return ((sx + bx - 1) / bx) * ((sy + 4 / bx - 1) / (4 / bx)); };
    const int64_t col = blocks(1), sq = blocks(2), row = blocks(4);
    shape = 3;
    if (sq < col) shape = 1;
    if (row < col && row < sq) shape = 2;
  }
  *bwx = shape == 1 ? 2 : (shape == 2 ? 4 : 1);
  *bwy = 4 / *bwx;
}

void raster_geometry(RasterQuery& a, int shape) {
  raster_block_shape(shape, a.W, a.H, &a.bwx, &a.bwy);
  a.tiles_x = (a.W + kSub * a.bwx - 1) / (kSub * a.bwx);
  a.tiles = a.tiles_x * ((a.H + kSub * a.bwy - 1) / (kSub * a.bwy));
  a.subs_x = (a.W + kSub - 1) / kSub;
  a.subs = raster_subtiles(a.W, a.H);
  a.pad = 0;
}

size_t raster_lds_bytes(int D, int S) {
  return (size_t)raster_table_slots(D) * sizeof(float4) +
         (size_t)4 * kFlush * 16 * sizeof(float) + (size_t)(D + 1) * sizeof(float);
}

int raster_max_samples() { return kMaxS; }

// S = 0 (the library's choice): the largest of 256, 128, 64 and 32 renders
// per block that still gives the launch (with the given block shape) at least
// 128 * S blocks (at 32
// renders per block, about two rounds of the blocks the chip holds at once).  Longer render runs per
// block amortise the per-block set-up (colour tables, target, cull
// rectangle); shorter ones keep small queries spread over all CUs.
int raster_auto_samples(int W, int H, uint64_t R, int shape) {
  int bwx, bwy;
  raster_block_shape(shape, W, H, &bwx, &bwy);
  const uint64_t tiles = (uint64_t)((W + kSub * bwx - 1) / (kSub * bwx)) *
                         (uint64_t)((H + kSub * bwy - 1) / (kSub * bwy));
  for (int S = 256; S > 32; S /= 2)
    if (tiles * ((R + S - 1) / S) >= 128ull * (uint64_t)S) return S;
  return 32;
}

void launch_raster_loss(hipStream_t st, const DiskScene& s, const float4* rec, uint64_t R,
                        int S, int shape, const RasterExact& ex, float* partial, const int* skip) {
  if (S <= 0) S = raster_auto_samples(s.W, s.H, R, shape);
  if (S > kMaxS) S = kMaxS;
  RasterQuery a;
  a.W = s.W; a.H = s.H; a.C = s.C; a.D = s.D; a.S = S;
  raster_geometry(a, shape);
  const int tiles = a.tiles;
  const uint64_t chunks = (R + S - 1) / S;
  const size_t lds = raster_lds_bytes(s.D, S);
  // grid: 8 XCD lanes x tiles x ceil(chunks / 8); launched in slices that keep
  // the block count within the grid limit
  const uint64_t per_xcd = (chunks + 7) / 8;
  const uint64_t max_rows = (1ull << 30) / (8ull * (uint64_t)tiles);
  for (uint64_t row0 = 0; row0 < per_xcd; row0 += max_rows) {
    const uint64_t rows = umin64(max_rows, per_xcd - row0);
    const uint64_t sub_chunks = umin64(chunks - row0 * 8, rows * 8);
    const uint64_t r_base = row0 * 8 * (uint64_t)S;
    a.rec = rec + r_base * (uint64_t)s.D;
    a.target = s.target;
    a.colors = s.colors;
    a.partial = partial;
    a.R = umin64(R - r_base, sub_chunks * (uint64_t)S);
    a.r_base = r_base;
    a.ex = ex;
    a.skip = skip;
    const dim3 grid((unsigned)(8 * tiles * rows));
#define HR_RASTER(CC, ONE) \
  hipLaunchKernelGGL((k_raster_loss<CC, ONE>), grid, dim3(256), lds, st, a, sub_chunks)
    const bool one = s.D <= 64;
    switch (s.C) {
      case 1: if (one) HR_RASTER(1, true); else HR_RASTER(1, false); break;
      case 2: if (one) HR_RASTER(2, true); else HR_RASTER(2, false); break;
      case 3: if (one) HR_RASTER(3, true); else HR_RASTER(3, false); break;
      default: if (one) HR_RASTER(4, true); else HR_RASTER(4, false); break;
    }
#undef HR_RASTER
  }
}

void launch_render_disks(hipStream_t st, const DiskScene& s, const RasterExact& ex, float* image) {
  hipLaunchKernelGGL(k_render_disks, dim3((s.W + 63) / 64, s.H), dim3(64), 0, st, ex, s.colors,
                     s.W, s.H, s.C, s.D, image);
}

void launch_batch_records(hipStream_t st, const BatchTable* T, int blocks) {
  hipLaunchKernelGGL(k_batch_records, dim3(blocks), dim3(256), 0, st, T);
}
typedef void (*BatchRasterKernel)(const BatchTable*);
static BatchRasterKernel batch_raster_kernel(int cls) {
  switch (cls) {
    case 0: return k_batch_raster<1, true>;
    case 1: return k_batch_raster<1, false>;
    case 2: return k_batch_raster<2, true>;
    case 3: return k_batch_raster<2, false>;
    case 4: return k_batch_raster<3, true>;
    case 5: return k_batch_raster<3, false>;
    case 6: return k_batch_raster<4, true>;
    default: return k_batch_raster<4, false>;
  }
}
// classes 8.. are the HVP render pairs (hr_edges.hip), by channel count
void launch_batch_raster(hipStream_t st, const BatchTable* T, int cls, int blocks, size_t lds) {
  if (raster_is_pair_class(cls)) {
    launch_batch_dloss(st, T, cls, blocks, lds);
    return;
  }
  hipLaunchKernelGGL(batch_raster_kernel(cls), dim3(blocks), dim3(256), lds, st, T);
}
int batch_raster_blocks_per_cu(int cls, size_t lds) {
  if (raster_is_pair_class(cls)) return batch_dloss_blocks_per_cu(cls, lds);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_raster_kernel(cls), 256, lds) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace hr
