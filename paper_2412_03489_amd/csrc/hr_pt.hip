// hr_pt.hip -- fused path tracer + MSE for the path-traced scene.
//
// Light transport (section "Background": Monte Carlo integration of the
// rendering equation with standard light and BRDF sampling): diffuse spheres
// on the plane y = 0, one square light facing -y; per path a jittered pinhole
// camera ray; emission only when the camera ray sees the light; next-event
// estimation to a uniform point on the light at the first and second surface
// hits; one cosine-weighted bounce; black background; no Russian roulette.
//
// Work decomposition: block = 16x16 pixel tile (one pixel per thread) x S
// draws; per draw all its renders (antithetic pair, HVP shifts) reuse the
// same pixel randomness and camera ray (common random numbers), so the Philox
// words and the primary ray are generated once per (pixel, spp) and traced
// against each render's light/sphere placement.  Loss partials per
// (render, tile) as in the rasteriser.
//
// Arithmetic: FP32 with the hardware's one-instruction reciprocal, square
// root, reciprocal square root and sine/cosine (the bounce angle is 2 pi u,
// and the hardware sine takes its argument in revolutions), within a few ulp;
// the path semantics are those of the FP64 reference.  Reciprocals of the
// sphere radii and the light's Le side^2 / pi are precomputed per scene.
#include <cstring>

#include "hr_device.h"
#include "hr_kernels.h"

namespace hr {

namespace {

constexpr int kPtTile = 16;
constexpr int kMaxSpheres = 16;
constexpr int kPtMaxS = 32;
constexpr float kEps = 1e-4f;
constexpr float kTmin = 1e-6f;

struct PTConst {
  float eye[3], fwd[3], right[3], up[3];
  float sx_scale, sy_scale;        // tan(vfov/2) * aspect, tan(vfov/2)
  float side, Le, ground[3];
  int ns, W, H, spp;
  float sph[kMaxSpheres][7];       // centre[3], radius, albedo[3]; centre of 0 from theta
  float inv_r[kMaxSpheres];        // 1 / radius
  float k_nee;                     // Le side^2 / pi
};

__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }

struct V3 { float x, y, z; };
__host__ __device__ __forceinline__ V3 v3(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(V3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ float dot3(V3 a, V3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }

struct Placement { V3 light, s0; };

template <class Consts>
__device__ __forceinline__ V3 sph_c(const Consts& P, const Placement& pl, int i) {
  return i == 0 ? pl.s0 : v3(P.sph[i][0], P.sph[i][1], P.sph[i][2]);
}

// ray/sphere: quadratic t^2 + 2 b t + c = 0 with |d| = 1; discriminant in the
// form r^2 - |oc - b d|^2, which keeps FP32 digits for distant spheres
__device__ __forceinline__ float hit_sphere(V3 o, V3 d, V3 c, float r) {
  const V3 oc = o - c;
  const float b = dot3(oc, d);
  const V3 l = oc - d * b;
  const float disc = fmaf(r, r, -dot3(l, l));
  if (disc < 0.0f) return -1.0f;
  const float sq = __builtin_amdgcn_sqrtf(disc);
  float t = -b - sq;
  if (!(t > kTmin)) t = -b + sq;
  return t > kTmin ? t : -1.0f;
}

// closest hit: -1 none, 0..ns-1 sphere, ns plane, ns+1 light
template <class Consts>
__device__ int intersect(const Consts& P, const Placement& pl, V3 o, V3 d, float& tb) {
  int id = -1;
  float best = 3.0e38f;
  for (int i = 0; i < P.ns; ++i) {
    const float t = hit_sphere(o, d, sph_c(P, pl, i), P.sph[i][3]);
    if (t > 0.0f && t < best) { best = t; id = i; }
  }
  if (d.y != 0.0f) {
    const float idy = rcp_f(d.y);
    const float t = -o.y * idy;
    if (t > kTmin && t < best) { best = t; id = P.ns; }
    const float tl = (pl.light.y - o.y) * idy;
    if (tl > kTmin && tl < best) {
      const V3 p = o + d * tl;
      const float half = 0.5f * P.side;
      if (fabsf(p.x - pl.light.x) <= half && fabsf(p.z - pl.light.z) <= half) { best = tl; id = P.ns + 1; }
    }
  }
  tb = best;
  return id;
}

// The part of a camera ray's closest hit that every render of a draw shares:
// spheres 1.. and the plane (the renders differ only in sphere 0 and the
// light).  Scanned in the same order and with the same strict comparisons as
// intersect(), so that camera_hit() below returns exactly what intersect()
// would.
struct CamHit {
  float t;
  int id;
};

template <class Consts>
__device__ __forceinline__ CamHit camera_common(const Consts& P, V3 o, V3 d) {
  int id = -1;
  float best = 3.0e38f;
  for (int i = 1; i < P.ns; ++i) {
    const float t = hit_sphere(o, d, v3(P.sph[i][0], P.sph[i][1], P.sph[i][2]), P.sph[i][3]);
    if (t > 0.0f && t < best) { best = t; id = i; }
  }
  if (d.y != 0.0f) {
    const float t = -o.y * rcp_f(d.y);
    if (t > kTmin && t < best) { best = t; id = P.ns; }
  }
  return {best, id};
}

// intersect() of a camera ray from the shared part: sphere 0 is scanned first
// there, so it keeps a tie (a later candidate must be strictly closer); the
// light is tested last with a strict comparison, as there.
template <class Consts>
__device__ __forceinline__ int camera_hit(const Consts& P, const Placement& pl, V3 o, V3 d,
                                          CamHit c, float& tb) {
  int id = c.id;
  float best = c.t;
  if (P.ns > 0) {
    const float t0 = hit_sphere(o, d, pl.s0, P.sph[0][3]);
    if (t0 > 0.0f && t0 <= best) { best = t0; id = 0; }
  }
  if (d.y != 0.0f) {
    const float idy = rcp_f(d.y);
    const float tl = (pl.light.y - o.y) * idy;
    if (tl > kTmin && tl < best) {
      const V3 p = o + d * tl;
      const float half = 0.5f * P.side;
      if (fabsf(p.x - pl.light.x) <= half && fabsf(p.z - pl.light.z) <= half) { best = tl; id = P.ns + 1; }
    }
  }
  tb = best;
  return id;
}

template <class Consts>
__device__ bool occluded(const Consts& P, const Placement& pl, V3 o, V3 d, float dist) {
  // every blocker is tested (no per-lane early exit: the wave would run on
  // until its last lane finished anyway)
  const float tmax = dist - kEps;
  bool hit = false;
  for (int i = 0; i < P.ns; ++i) {
    const float t = hit_sphere(o, d, sph_c(P, pl, i), P.sph[i][3]);
    hit = hit || (t > 0.0f && t < tmax);
  }
  if (d.y != 0.0f) {
    const float t = -o.y * rcp_f(d.y);
    hit = hit || (t > kTmin && t < tmax);
  }
  return hit;
}

// Le cos_x cos_l A / (pi d^2) for a uniform light point, visibility included
template <class Consts>
__device__ float nee(const Consts& P, const Placement& pl, V3 o, V3 n, float u1, float u2) {
  const V3 y = v3(pl.light.x + (u1 - 0.5f) * P.side, pl.light.y, pl.light.z + (u2 - 0.5f) * P.side);
  const V3 wv = y - o;
  const float d2 = dot3(wv, wv);
  const float idist = __builtin_amdgcn_rsqf(d2);
  const float dist = d2 * idist;
  const V3 wi = wv * idist;
  const float cx = dot3(n, wi), cl = wi.y;
  if (!(cx > 0.0f) || !(cl > 0.0f)) return 0.0f;
  if (occluded(P, pl, o, wi, dist)) return 0.0f;
  return P.k_nee * cx * cl * (idist * idist);
}

template <class Consts>
__device__ __forceinline__ void surface(const Consts& P, const Placement& pl, int id, V3 x, V3& n,
                                        V3& alb) {
  if (id < P.ns) {
    n = (x - sph_c(P, pl, id)) * P.inv_r[id];
    alb = v3(P.sph[id][4], P.sph[id][5], P.sph[id][6]);
  } else {
    n = v3(0.0f, 1.0f, 0.0f);
    alb = v3(P.ground[0], P.ground[1], P.ground[2]);
  }
}

// radiance of one path whose camera ray from `eye` along d first hits `id` at
// distance t; u[0..1] jitter (used by the caller), u[2..3] light sample at
// hit 1, u[4..5] bounce, u[6..7] light sample at hit 2
template <class Consts>
__device__ V3 radiance_from(const Consts& P, const Placement& pl, V3 eye, V3 d, int id, float t,
                            const float* u) {
  if (id < 0) return v3(0.f, 0.f, 0.f);
  if (id == P.ns + 1) return d.y > 0.0f ? v3(P.Le, P.Le, P.Le) : v3(0.f, 0.f, 0.f);
  const V3 x = eye + d * t;
  V3 n, alb;
  surface(P, pl, id, x, n, alb);
  const V3 o1 = x + n * kEps;
  const float e1 = nee(P, pl, o1, n, u[2], u[3]);
  V3 L = alb * e1;
  // cosine-weighted direction (Malley) in the basis of Duff et al. 2017
  const float rr = __builtin_amdgcn_sqrtf(u[4]);
  const float sgn = copysignf(1.0f, n.z);
  const float a = -rcp_f(sgn + n.z);   // |sgn + n.z| >= 1
  const float bb = n.x * n.y * a;
  const V3 b1 = v3(1.0f + sgn * n.x * n.x * a, sgn * bb, -sgn * n.x);
  const V3 b2 = v3(bb, sgn + n.y * n.y * a, -n.y);
  // angle 2 pi u[5]: the hardware sine and cosine take revolutions
  const float sp = __builtin_amdgcn_sinf(u[5]), cp = __builtin_amdgcn_cosf(u[5]);
  const V3 dir = b1 * (rr * cp) + b2 * (rr * sp) + n * __builtin_amdgcn_sqrtf(1.0f - u[4]);
  float t2;
  const int id2 = intersect(P, pl, o1, dir, t2);
  if (id2 < 0 || id2 == P.ns + 1) return L;
  const V3 x2 = o1 + dir * t2;
  V3 n2, alb2;
  surface(P, pl, id2, x2, n2, alb2);
  const V3 o2 = x2 + n2 * kEps;
  const float e2 = nee(P, pl, o2, n2, u[6], u[7]);
  L = L + v3(alb.x * alb2.x, alb.y * alb2.y, alb.z * alb2.z) * e2;
  return L;
}

template <class Consts>
__device__ V3 radiance(const Consts& P, const Placement& pl, V3 eye, V3 d, const float* u) {
  float t;
  const int id = intersect(P, pl, eye, d, t);
  return radiance_from(P, pl, eye, d, id, t, u);
}

__device__ __forceinline__ void path_uniforms(uint64_t seed, uint32_t s, uint32_t pix, int k,
                                              float* u) {
  const u32x4 wa = philox_seeded(seed, s, pix, (uint32_t)(16 * k + 0), kTagPixel);
  const u32x4 wb = philox_seeded(seed, s, pix, (uint32_t)(16 * k + 1), kTagPixel);
  u[0] = u01_f(wa.x); u[1] = u01_f(wa.y); u[2] = u01_f(wa.z); u[3] = u01_f(wa.w);
  u[4] = u01_f(wb.x); u[5] = u01_f(wb.y); u[6] = u01_f(wb.z); u[7] = u01_f(wb.w);
}

template <class Consts>
__device__ __forceinline__ V3 camera_dir(const Consts& P, int x, int y, float jx, float jy) {
  const float sx = (2.0f * ((float)x + jx) * rcp_f((float)P.W) - 1.0f) * P.sx_scale;
  const float sy = (1.0f - 2.0f * ((float)y + jy) * rcp_f((float)P.H)) * P.sy_scale;
  const V3 f = v3(P.fwd[0], P.fwd[1], P.fwd[2]);
  const V3 r = v3(P.right[0], P.right[1], P.right[2]);
  const V3 up = v3(P.up[0], P.up[1], P.up[2]);
  const V3 d = f + r * sx + up * sy;
  return d * __builtin_amdgcn_rsqf(dot3(d, d));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One block's work: draws [d0, d0 + nd) of one query on one 16x16 tile,
// all NR renders of each draw.  Shared by the per-query and the batch kernel.
template <int NR, class Consts>
__device__ __forceinline__ void pt_block(const Consts& P, const double* __restrict__ theta,
                                         const double* __restrict__ tau,
                                         const double* __restrict__ u,
                                         const float* __restrict__ target, const EstShape& e,
                                         int tiles_x, int tiles, int tile, uint64_t d0, int nd,
                                         float* __restrict__ partial, float (*s_part)[4]) {
  __syncthreads();   // the previous work item's readers of LDS are done
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = (tile % tiles_x) * kPtTile + (threadIdx.x & 15);
  const int y = (tile / tiles_x) * kPtTile + (threadIdx.x >> 4);
  const bool valid = x < P.W && y < P.H;
  const uint32_t pix = (uint32_t)(y * P.W + x);
  float T[3] = {0.f, 0.f, 0.f};
  if (valid)
    for (int c = 0; c < 3; ++c) T[c] = target[(size_t)pix * 3 + c];
  const V3 eye = v3(P.eye[0], P.eye[1], P.eye[2]);
  const float inv_spp = 1.0f / (float)P.spp;

  for (int dd = 0; dd < nd; ++dd) {
    const uint64_t sidx = d0 + dd;
    const uint32_t s = (uint32_t)(sidx % e.N);
    const double* t = tau + sidx * (uint64_t)e.n;
    Placement pl[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
      const int ai = rr / e.NH, sh = rr % e.NH;
      const double a = ai == 0 ? 1.0 : -1.0;
      const double shift = sh == 0 ? e.h : -e.h;
      float q[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        double base = theta[k];
        if (e.NH == 2) base = base + shift * u[k];
        q[k] = (float)(base - a * t[k]);
      }
      pl[rr].light = v3(q[0], q[1], q[2]);
      pl[rr].s0 = v3(q[3], q[4], q[5]);
    }
    float acc[NR][3];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) acc[rr][0] = acc[rr][1] = acc[rr][2] = 0.f;
    if (valid) {
      for (int k = 0; k < P.spp; ++k) {
        float uu[8];
        path_uniforms(e.seed, s, pix, k, uu);
        const V3 d = camera_dir(P, x, y, uu[0], uu[1]);
        // the camera ray's hits on what the renders share, found once
        const CamHit ch = camera_common(P, eye, d);
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
          float t;
          const int id = camera_hit(P, pl[rr], eye, d, ch, t);
          const V3 L = radiance_from(P, pl[rr], eye, d, id, t, uu);
          acc[rr][0] += L.x; acc[rr][1] += L.y; acc[rr][2] += L.z;
        }
      }
    }
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
      float ev = 0.0f;
      if (valid)
        for (int c = 0; c < 3; ++c) {
          const float df = acc[rr][c] * inv_spp - T[c];
          ev = fmaf(df, df, ev);
        }
      ev = wave_sum(ev);
      if (lane == 0) s_part[dd * NR + rr][wave] = ev;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nd * NR; i += blockDim.x) {
    const float v = ((s_part[i][0] + s_part[i][1]) + s_part[i][2]) + s_part[i][3];
    partial[part_index(d0 * (uint64_t)NR + (uint64_t)i, (uint64_t)tile, (uint64_t)tiles)] = v;
  }
}

typedef const PTConst __attribute__((address_space(4))) ConstPT;

// The scene's constants are read from device memory through the constant
// address space: scalar loads on use, and no private copy (a by-value
// argument passed by reference to the tracing routines would be copied to
// scratch).
// Two renders per draw (a Hessian or gradient with antithetic pairs): at least
// 6 waves per SIMD (80 VGPRs, a few bytes of spills outside the path loop)
// are 3% faster than the 5 the compiler picks by itself; 7 spill too much.
template <int NR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NR == 2 ? 6 : 1)))
void k_pt_loss(const PTConst* ptc, const double* __restrict__ theta,
               const double* __restrict__ tau,
               const double* __restrict__ u,
               const float* __restrict__ target, EstShape e,
               int S, int tiles_x, int tiles, uint64_t draw0,
               uint64_t chunks, float* __restrict__ partial) {
  __shared__ float s_part[kPtMaxS * NR][4];
  if (e.skip && *e.skip) return;
  // XCD-aware order as in the rasteriser
  const uint64_t b = blockIdx.x;
  const uint64_t xcd = b & 7u, j = b >> 3;
  const uint64_t chunk = (j / (uint64_t)tiles) * 8u + xcd;
  const int tile = (int)(j % (uint64_t)tiles);
  if (chunk >= chunks) return;
  const uint64_t total = e.streams * e.N;
  const uint64_t d0 = draw0 + chunk * (uint64_t)S;
  const int nd = (int)min((uint64_t)S, total - d0);
  ConstPT& P = *(ConstPT*)ptc;
  pt_block<NR>(P, theta, tau, u, target, e, tiles_x, tiles, tile, d0, nd, partial, s_part);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Persistent path tracer over eight work queues (same scheme as the
// persistent rasteriser: item = (query, chunk of S draws, 16x16 tile)); one
// kernel per number of renders per draw, so each keeps the register budget of
// the per-query kernel.  Query constants are read through the constant
// address space (the batch never writes them), as kernel arguments are.
typedef const PTConst __attribute__((address_space(4))) ConstPT;

template <int NR>
__global__ __launch_bounds__(256) void k_batch_pt(const BatchTable* __restrict__ T) {
  __shared__ float s_part[kPtMaxS * NR][4];
  __shared__ unsigned long long s_item;
  const WorkQueues& W = T->pt[NR == 1 ? 0 : (NR == 2 ? 1 : 2)];
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
    __syncthreads();
    while (it < nitems) {
      // the next item is claimed before this one's work (as in the rasteriser)
      unsigned long long next = 0;
      if (threadIdx.x == 0) next = atomicAdd(&W.ctr[x], 1ull);
      uint64_t lo = sb, hi = se - 1;
      while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (uniform64(W.seg[mid].item0) <= it) lo = mid; else hi = mid - 1;
      }
      const WorkSeg sg = uniform_copy(&W.seg[lo]);
      const BatchQuery& Q = T->q[sg.q];
      const EstShape e = uniform_copy(&Q.e);
      const uint64_t qp[4] = {uniform64((uint64_t)Q.theta), uniform64((uint64_t)Q.tau),
                              uniform64((uint64_t)Q.u), uniform64((uint64_t)Q.pt_target)};
      float* partial = (float*)uniform64((uint64_t)Q.partial);
      const int S = __builtin_amdgcn_readfirstlane(Q.pt_S);
      const int tiles_x = __builtin_amdgcn_readfirstlane(Q.pt_tiles_x);
      const int tiles = __builtin_amdgcn_readfirstlane(Q.pt_tiles);
      ConstPT& P = *(ConstPT*)uniform64((uint64_t)Q.ptc);
      const uint64_t l = it - sg.item0;
      const uint64_t chunk = (uint64_t)sg.c0 + 8u * (l / (uint64_t)sg.tiles);
      const int tile = (int)(l % (uint64_t)sg.tiles);
      const uint64_t d0 = chunk * (uint64_t)S;
      const int nd = (int)min((uint64_t)S, e.streams * e.N - d0);
      pt_block<NR>(P, (const double*)qp[0], (const double*)qp[1], (const double*)qp[2],
                   (const float*)qp[3], e, tiles_x, tiles, tile, d0, nd, partial, s_part);
      if (threadIdx.x == 0) s_item = next;
      __syncthreads();
      it = uniform64(s_item);
      __syncthreads();
    }
  }
}

__global__ void k_pt_render(PTConst P, Placement pl, uint64_t seed, uint32_t s, int spp,
                            float* __restrict__ image) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= P.W || y >= P.H) return;
  const uint32_t pix = (uint32_t)(y * P.W + x);
  const V3 eye = v3(P.eye[0], P.eye[1], P.eye[2]);
  float acc[3] = {0.f, 0.f, 0.f};
  for (int k = 0; k < spp; ++k) {
    float uu[8];
    path_uniforms(seed, s, pix, k, uu);
    const V3 d = camera_dir(P, x, y, uu[0], uu[1]);
    const V3 L = radiance(P, pl, eye, d, uu);
    acc[0] += L.x; acc[1] += L.y; acc[2] += L.z;
  }
  for (int c = 0; c < 3; ++c) image[(size_t)pix * 3 + c] = acc[c] / (float)spp;
}

PTConst make_const(const PTScene& s, int spp) {
  PTConst P{};
  const float* d = s.desc;   // host FP32 copy of the description + derived camera
  for (int i = 0; i < 3; ++i) {
    P.eye[i] = d[i];
    P.fwd[i] = d[12 + i];
    P.right[i] = d[15 + i];
    P.up[i] = d[18 + i];
  }
  P.sx_scale = d[21];
  P.sy_scale = d[22];
  P.side = d[7];
  P.Le = d[8];
  P.ground[0] = d[9]; P.ground[1] = d[10]; P.ground[2] = d[11];
  P.ns = s.nspheres;
  P.W = s.W; P.H = s.H; P.spp = spp;
  for (int i = 0; i < s.nspheres && i < kMaxSpheres; ++i) {
    for (int k = 0; k < 7; ++k) P.sph[i][k] = d[23 + 7 * i + k];
    P.inv_r[i] = 1.0f / P.sph[i][3];
  }
  P.k_nee = (float)((double)P.Le * P.side * P.side / 3.14159265358979323846);
  return P;
}

}  // namespace

int pt_tiles(int W, int H) { return ((W + kPtTile - 1) / kPtTile) * ((H + kPtTile - 1) / kPtTile); }
int pt_tiles_x(int W) { return (W + kPtTile - 1) / kPtTile; }

void launch_pt_loss(hipStream_t st, const EstShape& e, const PTScene& s, const double* theta,
                    const double* tau, const double* u, int S, float* partial) {
  if (S <= 0 || S > kPtMaxS) S = 8;
  const PTConst* P = (const PTConst*)s.ptc;
  const int tiles_x = (s.W + kPtTile - 1) / kPtTile;
  const int tiles = pt_tiles(s.W, s.H);
  const uint64_t draws = e.streams * e.N;
  const uint64_t chunks = (draws + S - 1) / S;
  const uint64_t per_xcd = (chunks + 7) / 8;
  const uint64_t max_rows = (1ull << 30) / (8ull * (uint64_t)tiles);
  const int nr = e.A * e.NH;
  for (uint64_t row0 = 0; row0 < per_xcd; row0 += max_rows) {
    const uint64_t rows = umin64(max_rows, per_xcd - row0);
    const uint64_t draw0 = row0 * 8 * (uint64_t)S;
    const uint64_t sub_chunks = umin64(chunks - row0 * 8, rows * 8);
    const dim3 grid((unsigned)(8 * tiles * rows));
    if (nr == 1)
      hipLaunchKernelGGL(k_pt_loss<1>, grid, dim3(256), 0, st, P, theta, tau, u, s.target, e, S, tiles_x, tiles, draw0, sub_chunks, partial);
    else if (nr == 2)
      hipLaunchKernelGGL(k_pt_loss<2>, grid, dim3(256), 0, st, P, theta, tau, u, s.target, e, S, tiles_x, tiles, draw0, sub_chunks, partial);
    else
      hipLaunchKernelGGL(k_pt_loss<4>, grid, dim3(256), 0, st, P, theta, tau, u, s.target, e, S, tiles_x, tiles, draw0, sub_chunks, partial);
  }
}

void launch_pt_render(hipStream_t st, const PTScene& s, const double* theta, uint64_t seed,
                      uint32_t sidx, int spp, float* image) {
  const PTConst P = make_const(s, spp);
  Placement pl;
  pl.light = v3((float)theta[0], (float)theta[1], (float)theta[2]);
  pl.s0 = v3((float)theta[3], (float)theta[4], (float)theta[5]);
  hipLaunchKernelGGL(k_pt_render, dim3((s.W + 63) / 64, s.H), dim3(64), 0, st, P, pl, seed, sidx,
                     spp, image);
}

size_t pt_const_bytes() { return sizeof(PTConst); }

void pt_fill_const(const PTScene& s, void* host_out) {
  const PTConst P = make_const(s, s.spp);
  memcpy(host_out, &P, sizeof(PTConst));
}

void launch_batch_pt(hipStream_t st, const BatchTable* T, int nr, int blocks) {
  if (nr == 1) hipLaunchKernelGGL(k_batch_pt<1>, dim3(blocks), dim3(256), 0, st, T);
  else if (nr == 2) hipLaunchKernelGGL(k_batch_pt<2>, dim3(blocks), dim3(256), 0, st, T);
  else hipLaunchKernelGGL(k_batch_pt<4>, dim3(blocks), dim3(256), 0, st, T);
}

int batch_pt_blocks_per_cu(int nr) {
  int nb = 0;
  hipError_t e = nr == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_pt<1>, 256, 0)
                 : nr == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_pt<2>, 256, 0)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_pt<4>, 256, 0);
  if (e != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

int pt_max_samples() { return kPtMaxS; }

}  // namespace hr
