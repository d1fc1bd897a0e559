// hr_edges.hip -- the HVP's render pairs on disk scenes: loss differences
// summed along the disks' edges.
//
// The central difference of the HVP (section "Hessian-vector product") needs,
// per draw s and antithetic sign a, only f(theta + h u - a tau_s) -
// f(theta - h u - a tau_s).  The two scenes of such a pair differ by the
// shift 2 h u: with e = h (|u_xy| + |u_r|), the most a shift moves a disk's
// edge, a pixel at distance d from the midpoint disk's centre (theta - a
// tau_s) is covered by both shifted disks when d < r - e and by neither when
// d >= r + e.  Each disk's record carries the squared outer and inner radii
// (r + e)^2 and (r - e)^2, widened and narrowed by the FP32 error band, so
// that the FP32 tests d^2 < outer ("maybe") and d^2 < inner ("sure") decide
// those cases exactly.  A pixel contributes to the difference only if the
// top disk that may cover it lies above the top disk that surely covers it,
// and then that top "maybe" disk is not sure there: the pixel lies in that
// disk's ring inner <= d^2 < outer, and no disk above it may cover it.  So
// instead of visiting every pixel, a wave walks, for one pair, the rows of
// every disk's ring and tests only the pixel centres the ring can hold
// (about 2e wide: a few hundred pixels per pair where the image has 65536);
// a ring pixel whose disk is the top "maybe" one is decided exactly in FP64
// from theta, tau and u -- the definition's own arithmetic -- under both
// shifts, and contributes (I+ - T)^2 - (I- - T)^2 summed over the channels.
// Every other pixel has the same top disk under both shifts and contributes
// nothing.  The decisions are those of rendering both scenes pixel by pixel
// with exact coverage.
//
// Work decomposition: one wave per pair.  Lane k builds disk k's record and
// its FP64 parameters under both shifts in LDS, the disks whose outer boxes
// meet its own (the only ones that can cover a pixel of its ring), and its
// ring's rows; the waves then take (disk, row) items 64 at a time and queue
// the few pixel centres of each row's ring spans in LDS, one per lane per
// step (the spans hold hardly more pixels than the ring, about 1.01 per ring
// pixel); 64 queued pixels are tested and decided at a time, one per lane.
// Each lane sums its pixels' contributions in FP32 in queue order and
// the wave adds the 64 sums in FP64 in a fixed order, so the result does not
// depend on the launch shape or on the batch a query runs in.
#include "hr_device.h"
#include "hr_kernels.h"

namespace hr {

namespace {

constexpr int kEdgeDisks = 64;    // disks of a scene on this path: one per lane
constexpr int kEdgeQueue = 128;   // queued span pixels: fewer than 64 + one step's 64
// Absolute slack, in image units, on every bound derived from a record (row
// ranges, ring spans, box overlaps): far above the FP32 rounding of the bound
// computations, far below a pixel.
constexpr float kEdgeEps = 2e-5f;
// pixel centres of images with W + H up to this are tabulated in LDS per block
constexpr int kEdgeTab = 2048;
static_assert(kEdgeTab <= 2048 && kEdgeDisks <= 64, "a queued pixel packs x, y and k in 28 bits");

// Bit masks over the disks: 32-bit words up to 32 disks (single-instruction
// bit scans), else 64-bit
template <int MD> struct EdgeMask;
template <> struct EdgeMask<32> {
  typedef uint32_t T;
  __device__ static int low(T m) { return __builtin_ctz(m); }
  __device__ static int high(T m) { return 31 - __builtin_clz(m); }
};
template <> struct EdgeMask<64> {
  typedef unsigned long long T;
  __device__ static int low(T m) { return __builtin_ctzll(m); }
  __device__ static int high(T m) { return 63 - __builtin_clzll(m); }
};

// One wave's share of LDS, for scenes of at most MD disks (32 or 64)
template <int MD>
struct EdgeWave {
  float4 rec[MD];                     // midpoint disk: cx, cy, outer^2, inner^2 (-1: none)
  // the disk under +h (theta + h u - a tau_s) and under -h: cx, cy and r^2
  // (-1 where r <= 0: no pixel is covered)
  double pp[MD][3];
  double pm[MD][3];
  // disks whose outer boxes meet this disk's, per quadrant of its box that
  // they reach: [dx >= 0 | (dy >= 0) << 1] for a pixel at (dx, dy) from its
  // centre
  typename EdgeMask<MD>::T nbr[MD][4];
  float rad[MD];                      // outer radius (-1: none)
  int off[MD + 1];                    // its first (disk, row) item; off[D] = all items
  // queued pixel of a ring span: x | y << 11 | the ring's disk << 22 (W, H <
  // 2048)
  uint32_t q[kEdgeQueue];
};

// Disk k of pair p: its midpoint record and its FP64 parameters under both
// shifts, with the arithmetic of the per-render records and of the exact
// coverage test.
template <int MD>
__device__ __forceinline__ void edge_disk(const PairQuery& a, uint64_t p, int k, EdgeWave<MD>& L) {
  const int ppd = a.ppd;
  const int ai = a.A == 2 ? (int)(p & 1u) : 0;
  const uint64_t sidx = a.A == 2 ? p >> 1 : p;
  const double* t = a.tau + sidx * (uint64_t)a.n;
  const double sa = ai == 0 ? 1.0 : -1.0;
  double m[3] = {0.0, 0.0, 0.0}, vp[3], vm[3];
  for (int q = 0; q < ppd; ++q) {
    const int j = k * ppd + q;
    const double th = a.theta[j], uj = a.u[j], tj = t[j];
    m[q] = th - sa * tj;
    vp[q] = (th + a.h * uj) - sa * tj;
    vm[q] = (th + (-a.h) * uj) - sa * tj;
  }
  if (ppd != 3) vp[2] = vm[2] = (double)a.radius[k];
  L.pp[k][0] = vp[0];
  L.pp[k][1] = vp[1];
  L.pp[k][2] = vp[2] > 0.0 ? vp[2] * vp[2] : -1.0;
  L.pm[k][0] = vm[0];
  L.pm[k][1] = vm[1];
  L.pm[k][2] = vm[2] > 0.0 ? vm[2] * vm[2] : -1.0;
  const double rad = ppd == 3 ? m[2] : (double)a.radius[k];
  const double ux = a.u[k * ppd], uy = a.u[k * ppd + 1], ur = ppd == 3 ? a.u[k * ppd + 2] : 0.0;
  const double e = a.h * (sqrt(ux * ux + uy * uy) + fabs(ur));
  const double rp = rad + e, rm = rad - e;
  float4 out = make_float4((float)m[0], (float)m[1], -1.0f, -1.0f);
  if (rp > 0.0) {
    // the band at the larger radius also covers the smaller one
    const double band = ambiguity_band(m[0], m[1], rp);
    out.z = (float)((rp * rp + band) * 1.00001);
    if (rm > 0.0) out.w = (float)(rm * rm - band);
  }
  L.rec[k] = out;
  // the outer radius, by the hardware square root (within 1 ulp): the bounds
  // built on it carry kEdgeEps of slack
  L.rad[k] = out.z > 0.0f ? __builtin_amdgcn_sqrtf(out.z) : -1.0f;
}

// first row of a disk's ring (its outer box widened by kEdgeEps)
__device__ __forceinline__ int edge_row0(const float4& v, float R, int H) {
  return max(0, (int)floorf((v.y - R - kEdgeEps) * (float)H - 0.5f));
}

// Pixel centres tabulated in the block's LDS (W + H <= kEdgeTab; x-centres,
// then y): the FP32 ones of the per-render rasteriser, ((float)x + 0.5f) / W,
// and the FP64 ones of the exact test, (x + 0.5) / W.  The 32-disk layout
// keeps only the FP64 table and rounds it to FP32: both divisions round
// correctly, and a quotient (2i + 1) / 2n (n = W or H, n < 2^11) lies at
// least 2^-37 (relative) away from every FP32 rounding midpoint it does not
// equal (a midpoint has 25 significant bits), far beyond the FP64 rounding,
// so the rounded FP64 centre is the FP32 centre.
// The 64-disk layout keeps only the FP32 table and divides in FP64 where it
// needs the exact centre.
template <int MD>
struct EdgeCentres {
  const void* tab;
  int W, H;
  __device__ float fx(int x) const {
    return MD == 32 ? (float)((const double*)tab)[x] : ((const float*)tab)[x];
  }
  __device__ float fy(int y) const {
    return MD == 32 ? (float)((const double*)tab)[W + y] : ((const float*)tab)[W + y];
  }
  __device__ double dx(int x) const {
    return MD == 32 ? ((const double*)tab)[x] : ((double)x + 0.5) / (double)W;
  }
  __device__ double dy(int y) const {
    return MD == 32 ? ((const double*)tab)[W + y] : ((double)y + 0.5) / (double)H;
  }
};

// One pixel of a ring span of disk k: if it is in the ring, the top disk
// under each shift and the pixel's (I+ - T)^2 - (I- - T)^2 over the channels
// (0 if the pixel belongs to the ring of a disk above k, which counts it
// instead); 0 outside the ring.  The ring test is the FP32 test of every
// other "maybe" and "sure" decision, so each pixel is counted in at most one
// disk's ring.
template <int C, int MD>
__device__ __forceinline__ float edge_pixel(const PairQuery& a, const EdgeWave<MD>& L,
                                            const float4* s_col, const EdgeCentres<MD>& ct,
                                            int x, int y, int k) {
  typedef EdgeMask<MD> M;
  typedef typename M::T Mask;
  const float pxf = ct.fx(x), pyf = ct.fy(y);
  // a pixel of one of disk k's row spans: in its ring (inner <= d^2 <
  // outer), or contributing nothing here
  const float4 vk = L.rec[k];
  const float dxk = pxf - vk.x, dyk = pyf - vk.y;
  const float d2k = fmaf(dyk, dyk, dxk * dxk);
  if (!(d2k < vk.z) || d2k < vk.w) return 0.0f;
  // only the neighbours that reach the pixel's quadrant of disk k's box can
  // cover it
  const Mask nb = L.nbr[k][(dxk >= 0.0f ? 1 : 0) | (dyk >= 0.0f ? 2 : 0)];
  // a disk above k that may cover the pixel: the pixel is in that disk's ring
  // or inside it, and is counted there (or contributes nothing)
  Mask up = k < MD - 1 ? nb & (~Mask(0) << (k + 1)) : Mask(0);
  while (up) {
    const int j = M::low(up);
    up &= up - 1;
    const float4 v = L.rec[j];
    const float dx = pxf - v.x, dy = pyf - v.y;
    if (fmaf(dy, dy, dx * dx) < v.z) return 0.0f;
  }
  // the top disk below k that surely covers the pixel (-1: the background)
  const Mask below = nb & ((Mask(1) << k) - Mask(1));
  Mask dn = below;
  int ks = -1;
  while (dn) {
    const int j = M::high(dn);
    dn &= ~(Mask(1) << j);
    const float4 v = L.rec[j];
    const float dx = pxf - v.x, dy = pyf - v.y;
    if (fmaf(dy, dy, dx * dx) < v.w) { ks = j; break; }
  }
  // exact decisions, from k down: k first (it may cover the pixel), then the
  // disks between ks and k that may (their FP32 test against the outer
  // radius rules out the others for both shifts)
  const double pxd = ct.dx(x), pyd = ct.dy(y);
  int top_p = ks, top_m = ks;
  bool done_p = false, done_m = false;
  auto exact = [&](int j) {
    const double dxp = pxd - L.pp[j][0], dyp = pyd - L.pp[j][1];
    const double dxm = pxd - L.pm[j][0], dym = pyd - L.pm[j][1];
    if (!done_p && dxp * dxp + dyp * dyp < L.pp[j][2]) { top_p = j; done_p = true; }
    if (!done_m && dxm * dxm + dym * dym < L.pm[j][2]) { top_m = j; done_m = true; }
  };
  exact(k);
  Mask cand = ks < 0 ? below : below & ~((Mask(2) << ks) - Mask(1));
  while (cand != Mask(0) && !(done_p && done_m)) {
    const int j = M::high(cand);
    cand &= ~(Mask(1) << j);
    const float4 v = L.rec[j];
    const float dx = pxf - v.x, dy = pyf - v.y;
    if (!(fmaf(dy, dy, dx * dx) < v.z)) continue;   // neither shift covers
    exact(j);
  }
  if (top_p == top_m) return 0.0f;
  // colours: entry k + 1 is disk k, entry 0 the background
  const float4 cp = s_col[top_p + 1], cm = s_col[top_m + 1];
  const float ap[4] = {cp.x, cp.y, cp.z, cp.w}, am[4] = {cm.x, cm.y, cm.z, cm.w};
  const float* tg = a.target + ((size_t)y * a.W + x) * C;
  float acc = 0.0f;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const float t2 = 2.0f * tg[c];
    // (cp - T)^2 - (cm - T)^2 = (cp - cm)(cp + cm - 2T)
    acc = fmaf(ap[c] - am[c], (ap[c] + am[c]) - t2, acc);
  }
  return acc;
}

// Pair p by one wave: f[p] = scale * (sum over the pair's pixels of the
// squared-error difference).
template <int C, int MD>
__device__ __forceinline__ void edge_pair(const PairQuery& a, uint64_t p, EdgeWave<MD>& L,
                                          const float4* s_col, const EdgeCentres<MD>& ct) {
  const int lane = threadIdx.x & 63;
  const int D = a.D, W = a.W, H = a.H;
  // lane k: disk k's record and parameters, and the number of its ring's rows
  int cnt = 0;
  if (lane < D) {
    edge_disk(a, p, lane, L);
    const float4 v = L.rec[lane];
    if (v.z > 0.0f) {
      const float R = L.rad[lane];
      const int y0 = edge_row0(v, R, H);
      const int y1 = min(H - 1, (int)ceilf((v.y + R + kEdgeEps) * (float)H - 0.5f));
      cnt = max(0, y1 - y0 + 1);
    }
  }
  // first item of each disk (exclusive prefix sum over the lanes)
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane < D) L.off[lane] = incl - cnt;
  if (lane == D - 1) L.off[D] = incl;
  const int total = __shfl(incl, 63, 64);
  __builtin_amdgcn_wave_barrier();
  // the disks whose outer boxes meet disk k's, per quadrant of disk k's box
  // that they reach (a disk that may cover a pixel at x >= cx_k reaches
  // cx_j + r_j + slack >= cx_k, and so on): up to 32 disks lanes k and
  // k + 32 test half of them each, else lane k tests all
  {
    typedef typename EdgeMask<MD>::T Mask;
    const bool halves = D <= 32;
    const int k = halves ? (lane & 31) : lane;
    const int j0 = halves && lane >= 32 ? (D + 1) / 2 : 0;
    const int j1 = halves && lane < 32 ? (D + 1) / 2 : D;
    Mask m[4] = {0, 0, 0, 0};
    if (k < D) {
      const float4 vk = L.rec[k];
      const float rk = L.rad[k];
      if (rk > 0.0f)
        for (int j = j0; j < j1; ++j) {
          const float4 vj = L.rec[j];
          const float rj = L.rad[j];
          const float reach = rj + rk + 2.0f * kEdgeEps;
          const bool meet = j != k && rj > 0.0f && fabsf(vj.x - vk.x) <= reach &&
                            fabsf(vj.y - vk.y) <= reach;
          const Mask bit = meet ? Mask(1) << j : Mask(0);
          const float rs = rj + 2.0f * kEdgeEps;
          const bool east = vj.x + rs >= vk.x, west = vj.x - rs <= vk.x;
          const bool north = vj.y + rs >= vk.y, south = vj.y - rs <= vk.y;
          m[0] |= west && south ? bit : Mask(0);
          m[1] |= east && south ? bit : Mask(0);
          m[2] |= west && north ? bit : Mask(0);
          m[3] |= east && north ? bit : Mask(0);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (halves) m[q] |= __shfl_xor(m[q], 32, 64);
      if (lane < D) L.nbr[lane][q] = m[q];
    }
  }
  __builtin_amdgcn_wave_barrier();

  float sum = 0.0f;           // this lane's contributions, in queue order
  uint32_t qlen = 0;          // wave-uniform queue length
  auto process = [&](int cnt_q) {
    float c = 0.0f;
    if (lane < cnt_q) {
      const uint32_t e = L.q[lane];
      c = edge_pixel<C, MD>(a, L, s_col, ct, (int)(e & 0x7ffu), (int)((e >> 11) & 0x7ffu),
                            (int)(e >> 22));
    }
    sum += c;
    // the rest of the queue to the front
    const int rest = (int)qlen - cnt_q;
    if (lane < rest) {
      const uint32_t e = L.q[cnt_q + lane];
      __builtin_amdgcn_wave_barrier();
      L.q[lane] = e;
    }
    qlen -= (uint32_t)cnt_q;
    __builtin_amdgcn_wave_barrier();
  };

  int kcur = 0;   // items are in disk order: a lane's disk only moves up
  for (int base = 0; base < total; base += 64) {
    const int it = base + lane;
    int x = 1, xe = 0, xc = 1, xd = 0, k = kcur;
    uint32_t yk = 0;   // the queued word's bits fixed by the item: y, k
    if (it < total) {
      while (L.off[k + 1] <= it) ++k;
      kcur = k;
      const float4 v = L.rec[k];
      const int y = edge_row0(v, L.rad[k], H) + (it - L.off[k]);
      yk = ((uint32_t)y << 11) | ((uint32_t)k << 22);
      const float dy = ct.fy(y) - v.y;
      const float dy2 = dy * dy;
      // |dx| < ro holds for every pixel with d^2 < outer on this row and
      // |dx| >= ri for every one with d^2 >= inner (slack: the FP32 rounding
      // of d^2 and of these bounds)
      const float slack = 0x1p-22f * (dy2 + v.z);
      const float ro = __builtin_amdgcn_sqrtf(fmaxf(v.z - dy2 + slack, 0.0f));
      const float i2 = v.w - dy2 - slack;
      const float ri = i2 > 0.0f ? __builtin_amdgcn_sqrtf(i2) : 0.0f;
      // centres in [cx - ro, cx - ri] and [cx + ri, cx + ro], each widened
      x = max(0, (int)ceilf((v.x - ro - kEdgeEps) * (float)W - 0.5f));
      xe = min(W - 1, (int)floorf((v.x - ri + kEdgeEps) * (float)W - 0.5f));
      xc = max(0, (int)ceilf((v.x + ri - kEdgeEps) * (float)W - 0.5f));
      xd = min(W - 1, (int)floorf((v.x + ro + kEdgeEps) * (float)W - 0.5f));
      if (xc <= xe) xc = xe + 1;   // no pixel is tested twice
      if (x > xe) { x = xc; xe = xd; xc = 1; xd = 0; }
    }
    // the spans' pixels queued one per lane per step (the spans hold hardly
    // more than the ring: the ring test comes with the decision), the queue
    // drained 64 at a time
    for (;;) {
      const bool act = x <= xe;
      const uint64_t b = __builtin_amdgcn_ballot_w64(act);
      if (b == 0ull) break;
      if (act) {
        const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)b, qlen));
        L.q[pos] = (uint32_t)x | yk;
      }
      qlen += (uint32_t)__builtin_popcountll(b);
      __builtin_amdgcn_wave_barrier();
      if (qlen >= 64) process(64);
      if (act) {
        ++x;
        if (x > xe) { x = xc; xe = xd; xc = 1; xd = 0; }
      }
    }
  }
  if (qlen > 0) process((int)qlen);
  // the 64 lane sums in FP64, in a fixed order
  double s = (double)sum;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) a.f[p] = s * a.scale;
  __builtin_amdgcn_wave_barrier();   // LDS of this pair read before the next pair's writes
}

// the block's colour table: entry 0 the background, entry k + 1 disk k
__device__ __forceinline__ void edge_colours(const PairQuery& a, float4* s_col) {
  for (int t = threadIdx.x; t <= a.D; t += blockDim.x) {
    float cc[4] = {0.f, 0.f, 0.f, 0.f};
    if (t > 0)
      for (int c = 0; c < a.C; ++c) cc[c] = a.colors[(size_t)(t - 1) * a.C + c];
    s_col[t] = make_float4(cc[0], cc[1], cc[2], cc[3]);
  }
}

// the block's pixel-centre table (see EdgeCentres) at tab
template <int MD>
__device__ __forceinline__ EdgeCentres<MD> edge_centres(int W, int H, void* tab) {
  for (int t = threadIdx.x; t < W + H; t += blockDim.x) {
    const int i = t < W ? t : t - W, n = t < W ? W : H;
    if (MD == 32) ((double*)tab)[t] = ((double)i + 0.5) / (double)n;
    else ((float*)tab)[t] = ((float)i + 0.5f) / (float)n;
  }
  EdgeCentres<MD> ct;
  ct.tab = tab;
  ct.W = W;
  ct.H = H;
  return ct;
}

// LDS layout of a block: colour table, four waves' shares, pixel centres
// (FP64 with up to 32 disks, else FP32)
template <int MD>
__host__ __device__ inline size_t edge_lds_bytes(int W, int H) {
  static_assert(((MD + 1) * sizeof(float4) + 4 * sizeof(EdgeWave<MD>)) % 8 == 0,
                "the centre table starts 8-byte aligned");
  return (size_t)(MD + 1) * sizeof(float4) + 4 * sizeof(EdgeWave<MD>) +
         (size_t)(W + H) * (MD == 32 ? sizeof(double) : sizeof(float));
}

// Up to 32 disks the block's LDS (17.6 KB at 256 x 256) leaves room for 8
// blocks of four waves per CU (46 VGPRs, no spills); the kernel, latency-
// bound on its LDS and FP64 chains, ran faster with each step from 5 to 8
// waves per SIMD and no faster at 9 (a layout without the radius table).  The 7 asked for keeps the register
// budget from dropping below 72.  With 64 disks the LDS allows 5.
template <int C, int MD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MD == 32 ? 7 : 1)))
void k_raster_dloss(PairQuery a) {
  extern __shared__ float4 smem[];
  if (a.skip && *a.skip) return;
  float4* s_col = smem;
  EdgeWave<MD>* s_w = (EdgeWave<MD>*)(smem + MD + 1);
  edge_colours(a, s_col);
  const EdgeCentres<MD> ct = edge_centres<MD>(a.W, a.H, s_w + 4);
  __syncthreads();
  // one pair per wave, no loop: values set up for the pair die with it
  // instead of living across a loop (which costs spilled registers)
  const int wave = threadIdx.x >> 6;
  const uint64_t p = ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * 4 + wave;
  if (p < a.L) edge_pair<C, MD>(a, p, s_w[wave], s_col, ct);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Persistent form over the eight work queues of one pair class (channel
// count and LDS layout; the 32-disk layout's queues hold scenes of up to 32
// disks only): an item is (query, chunk of S pairs); blocks start on the
// queue of their XCD, claim items by one atomic increment each (the next one
// before working on the current one), move on to the other queues when
// theirs is empty, and leave after seeing all eight exhausted.
// Registers for 5 waves per SIMD with either layout: the LDS of the largest
// query of the batch decides the blocks per CU, and with 32 disks asking for
// 7 (more spills) or 6 was no faster on the 64 uneven instances.
template <int C, int MD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
void k_batch_dloss(const BatchTable* __restrict__ T) {
  extern __shared__ float4 smem[];
  __shared__ unsigned long long s_item;
  const WorkQueues& W = T->raster[raster_pair_class(C, MD)];
  const int home = blockIdx.x & 7;
  uint64_t all = 0;
  for (int x = 0; x < 8; ++x) all += W.items[x];
  if (all == 0) return;   // nothing of this kind in the batch
  float4* s_col = smem;
  EdgeWave<MD>* s_w = (EdgeWave<MD>*)(smem + MD + 1);
  const int wave = threadIdx.x >> 6;
  for (int kq = 0; kq < 8; ++kq) {
    const int x = (home + kq) & 7;
    const uint64_t nitems = W.items[x];
    const uint64_t sb = W.seg_off[x], se = W.seg_off[x + 1];
    if (threadIdx.x == 0) s_item = atomicAdd(&W.ctr[x], 1ull);
    __syncthreads();
    uint64_t it = uniform64(s_item);
    __syncthreads();   // every thread has read s_item before it is reused
    while (it < nitems) {
      unsigned long long next = 0;
      if (threadIdx.x == 0) next = atomicAdd(&W.ctr[x], 1ull);
      uint64_t lo = sb, hi = se - 1;
      while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (uniform64(W.seg[mid].item0) <= it) lo = mid; else hi = mid - 1;
      }
      const WorkSeg sg = uniform_copy(&W.seg[lo]);
      const BatchQuery& Q = T->q[sg.q];
      PairQuery a;
      a.theta = (const double*)uniform64((uint64_t)Q.theta);
      a.tau = (const double*)uniform64((uint64_t)Q.tau);
      a.u = (const double*)uniform64((uint64_t)Q.u);
      a.radius = (const float*)uniform64((uint64_t)Q.ds.radius);
      a.colors = (const float*)uniform64((uint64_t)Q.ds.colors);
      a.target = (const float*)uniform64((uint64_t)Q.ds.target);
      a.f = (double*)uniform64((uint64_t)Q.f);
      a.W = __builtin_amdgcn_readfirstlane(Q.ds.W);
      a.H = __builtin_amdgcn_readfirstlane(Q.ds.H);
      a.C = C;
      a.D = __builtin_amdgcn_readfirstlane(Q.ds.D);
      a.ppd = __builtin_amdgcn_readfirstlane(Q.ds.ppd);
      a.n = __builtin_amdgcn_readfirstlane(Q.e.n);
      a.A = __builtin_amdgcn_readfirstlane(Q.e.A);
      a.h = Q.e.h;
      a.scale = Q.inv_count;
      a.L = uniform64(Q.e.L);
      a.S = __builtin_amdgcn_readfirstlane(Q.rq.S);
      a.skip = nullptr;
      const uint64_t chunk = (uint64_t)sg.c0 + 8u * (it - sg.item0);
      const uint64_t p0 = chunk * (uint64_t)a.S;
      const uint64_t p1 = umin64(p0 + (uint64_t)a.S, a.L);
      __syncthreads();   // the previous item's readers of the tables are done
      edge_colours(a, s_col);
      const EdgeCentres<MD> ct = edge_centres<MD>(a.W, a.H, s_w + 4);
      __syncthreads();
      for (uint64_t p = p0 + wave; p < p1; p += 4) edge_pair<C, MD>(a, p, s_w[wave], s_col, ct);
      if (threadIdx.x == 0) s_item = next;
      __syncthreads();
      it = uniform64(s_item);
      __syncthreads();
    }
  }
}

}  // namespace

// LDS of a pair query in the persistent kernel of its class (the layout by
// disk count, as raster_pair_class assigns it)
size_t raster_pair_lds_bytes(int W, int H, int D) {
  return D <= 32 ? edge_lds_bytes<32>(W, H) : edge_lds_bytes<kEdgeDisks>(W, H);
}

int raster_pair_max_side_sum() { return kEdgeTab; }

int raster_pair_max_disks() { return kEdgeDisks; }

template <int MD>
static void launch_dloss_md(hipStream_t st, const PairQuery& a) {
  const size_t lds = edge_lds_bytes<MD>(a.W, a.H);
  // one wave per pair: rows of up to 2^20 blocks
  const uint64_t blocks = std::max<uint64_t>((a.L + 3) / 4, 1);
  const uint64_t gx = umin64(blocks, 1ull << 20);
  const dim3 grid((unsigned)gx, (unsigned)((blocks + gx - 1) / gx));
  switch (a.C) {
    case 1: hipLaunchKernelGGL((k_raster_dloss<1, MD>), grid, dim3(256), lds, st, a); break;
    case 2: hipLaunchKernelGGL((k_raster_dloss<2, MD>), grid, dim3(256), lds, st, a); break;
    case 3: hipLaunchKernelGGL((k_raster_dloss<3, MD>), grid, dim3(256), lds, st, a); break;
    default: hipLaunchKernelGGL((k_raster_dloss<4, MD>), grid, dim3(256), lds, st, a); break;
  }
}

void launch_raster_dloss(hipStream_t st, const PairQuery& a) {
  // up to 32 disks: half the per-wave LDS, more blocks per CU
  if (a.D <= 32) launch_dloss_md<32>(st, a);
  else launch_dloss_md<kEdgeDisks>(st, a);
}

typedef void (*BatchDlossKernel)(const BatchTable*);
static BatchDlossKernel batch_dloss_kernel(int cls) {
  switch (cls) {
    case raster_pair_class(1, 64): return k_batch_dloss<1, 64>;
    case raster_pair_class(2, 64): return k_batch_dloss<2, 64>;
    case raster_pair_class(3, 64): return k_batch_dloss<3, 64>;
    case raster_pair_class(4, 64): return k_batch_dloss<4, 64>;
    case raster_pair_class(1, 32): return k_batch_dloss<1, 32>;
    case raster_pair_class(2, 32): return k_batch_dloss<2, 32>;
    case raster_pair_class(3, 32): return k_batch_dloss<3, 32>;
    default: return k_batch_dloss<4, 32>;
  }
}

void launch_batch_dloss(hipStream_t st, const BatchTable* T, int cls, int blocks, size_t lds) {
  hipLaunchKernelGGL(batch_dloss_kernel(cls), dim3(blocks), dim3(256), lds, st, T);
}

int batch_dloss_blocks_per_cu(int cls, size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_dloss_kernel(cls), 256, lds) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace hr
