// hr_estim.hip -- draws, analytic test scenes, lobe weights and accumulation.
//
// Estimator (sections "Gradients", "Hessians", "Hessian-vector product",
// "Aggregate" of Wang, Fischer, Ritschel 2025), for element m with kernel
// factor d_m (D kappa_m(tau) = d_m(tau) N(tau)):
//   est_m = 1/(A N) sum_s sum_a w_m(a tau_s) F(theta - a tau_s)
//   IS    : w_m = sgn(d_m) Z_m     AIS: w_m = d_m / q,  q = 1/K sum_k |d_k|/Z_k
//           (Hessian kernel, n^2 mixture: q = 1/n^2 sum_{i,j} |d_ij|/Z_ij)
//   GAUSS : w_m = d_m
// Gradient factors are odd in tau and Hessian factors even, so the antithetic
// partner's weight is -w or +w; per draw the renders collapse to one scalar F_s.
// Contributions c = d_m F_s / q are rounded to FP32 and summed per chunk of
// draws into positive and negative lobe sums with TwoSum compensation
// (or in FP64); the chunk sums are combined in fixed order in FP64.
#include "hr_device.h"
#include "hr_kernels.h"

namespace hr {

namespace {

constexpr double kPi = 3.14159265358979323846;

inline unsigned grid_for(uint64_t total, int block) {
  uint64_t g = (total + block - 1) / block;
  return (unsigned)(g > 65536u * 16u ? 65536u * 16u : (g == 0 ? 1 : g));
}

// draw component gid = (stream * N + s) * n + j.  The aggregate selector picks
// one of the K elements, or with mix_n2 one of the n^2 ordered pairs (i, j),
// drawn with the lobes of the element (min, max).
__device__ __forceinline__ void sample_one(int n, int K, int hessk, int mix_n2, int sampler,
                                           uint64_t N, uint64_t seed, double sg, uint64_t gid,
                                           double* __restrict__ tau) {
  const int j = (int)(gid % (uint64_t)n);
  const uint64_t sidx = gid / (uint64_t)n;
  const uint32_t stream = (uint32_t)(sidx / N);
  const uint32_t s = (uint32_t)(sidx % N);
  const uint32_t tag = per_element(sampler) ? stream : (sampler == kAIS ? kTagAIS : kTagGauss);
  const u32x4 w = philox_seeded(seed, s, (uint32_t)j, 0u, tag);
  int m = -1, i = -1, jj = -1;
  if (per_element(sampler)) m = (int)stream;
  if (sampler == kAIS) {
    const u32x4 ws = philox_seeded(seed, s, kDimSelect, 0u, tag);
    if (hessk && mix_n2) {
      const uint64_t nn = (uint64_t)n * (uint64_t)n;
      const int pair = (int)(((uint64_t)ws.x * nn) >> 32);
      i = pair / n;
      jj = pair % n;
    } else {
      m = (int)(((uint64_t)ws.x * (uint64_t)K) >> 32);
    }
  }
  if (m >= 0) {
    if (hessk) tri_ij(n, m, i, jj);
    else i = jj = m;
  }
  bool lg = false, ld = false;
  if (i >= 0) {
    if (!hessk) lg = (j == i);
    else if (i == jj) ld = (j == i);
    else lg = (j == i || j == jj);
  }
  double t;
  if (ld) {
    t = hdiag_lobe(w.z, sg);
  } else if (sampler == kFR22 && !lg) {
    t = 0.0;   // only the differentiated dimension is blurred
  } else {
    // the gradient lobe's Rayleigh magnitude and the Box-Muller radius share
    // one sqrt(-2 log x), so the lobe's lane does not run its own copy while
    // the rest of the wave waits: the same operations on the same operands as
    // grad_lobe and the Gaussian below
    const uint32_t wz = w.z;
    const bool lo = wz < 0x80000000u;
    const double x = lg ? fma((double)(lo ? wz : 0xFFFFFFFFu - wz), 0x1p-31, 0x1p-32)
                        : u01_d(w.x);
    const double rad = sqrt(-2.0 * log(x));
    t = lg ? (lo ? -sg : sg) * rad : sg * rad * cos(2.0 * kPi * u01_d(w.y));
  }
  tau[gid] = t;
}

// one thread per (stream, draw, dimension)
__global__ void k_sample(int n, int K, int hessk, int mix_n2, int sampler, uint64_t N,
                         uint64_t seed, double sg, uint64_t total, double* __restrict__ tau,
                         const int* skip) {
  if (skip && *skip) return;
  for (uint64_t gid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; gid < total;
       gid += (uint64_t)gridDim.x * blockDim.x)
    sample_one(n, K, hessk, mix_n2, sampler, N, seed, sg, gid, tau);
}

__device__ __forceinline__ void vnorm_block(int n, const double* __restrict__ v,
                                            double* __restrict__ u, double* __restrict__ vnorm,
                                            double* s_acc) {
  __syncthreads();
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) acc += v[j] * v[j];
  s_acc[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) s_acc[threadIdx.x] += s_acc[threadIdx.x + off];
    __syncthreads();
  }
  const double nv = sqrt(s_acc[0]);
  for (int j = threadIdx.x; j < n; j += blockDim.x) u[j] = nv > 0.0 ? v[j] / nv : 0.0;
  if (threadIdx.x == 0) *vnorm = nv;
}

// the draws of an HVP query, with |v| and v / |v| from block 0 first (one
// launch instead of two; the same arithmetic as the batch sampling phase)
__global__ __launch_bounds__(256) void k_sample_vnorm(int n, int K, int hessk, int mix_n2,
                                                      int sampler, uint64_t N, uint64_t seed,
                                                      double sg, uint64_t total,
                                                      double* __restrict__ tau,
                                                      const double* __restrict__ v,
                                                      double* __restrict__ u,
                                                      double* __restrict__ vnorm,
                                                      const int* skip) {
  __shared__ double s_acc[256];
  if (skip && *skip) return;
  if (blockIdx.x == 0) vnorm_block(n, v, u, vnorm, s_acc);
  for (uint64_t gid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; gid < total;
       gid += (uint64_t)gridDim.x * blockDim.x)
    sample_one(n, K, hessk, mix_n2, sampler, N, seed, sg, gid, tau);
}

// analytic scenes: render r in FP64
__device__ __forceinline__ void analytic_one(int kind, int n, const double* __restrict__ A,
                                             const double* __restrict__ b, double c, double s1,
                                             const double* __restrict__ theta,
                                             const double* __restrict__ tau,
                                             const double* __restrict__ u, int Aa, int NH,
                                             double h, uint64_t r, double* __restrict__ f) {
  const int sh = (int)(r % (uint64_t)NH);
  const uint64_t rem = r / (uint64_t)NH;
  const int ai = (int)(rem % (uint64_t)Aa);
  const uint64_t sidx = rem / (uint64_t)Aa;
  const double* t = tau + sidx * (uint64_t)n;
  const double a = ai == 0 ? 1.0 : -1.0;
  const double shift = sh == 0 ? h : -h;
  auto P = [&](int j) {
    double base = theta[j];
    if (NH == 2) base = base + shift * u[j];
    return base - a * t[j];
  };
  double val;
  if (kind == 0) {
    val = c;
    for (int i = 0; i < n; ++i) {
      const double pi = P(i);
      val += b[i] * pi;
      for (int j = 0; j < n; ++j) val += 0.5 * pi * A[i * n + j] * P(j);
    }
  } else {
    double r2 = 0.0;
    for (int i = 0; i < n; ++i) {
      const double pi = P(i);
      r2 += pi * pi;
    }
    val = -pow(2.0 * kPi * s1 * s1, -0.5 * n) * exp(-r2 / (2.0 * s1 * s1));
  }
  f[r] = val;
}

__global__ void k_analytic(int kind, int n, const double* __restrict__ A,
                           const double* __restrict__ b, double c, double s1,
                           const double* __restrict__ theta, const double* __restrict__ tau,
                           const double* __restrict__ u, int Aa, int NH, double h, uint64_t R,
                           double* __restrict__ f, const int* skip) {
  if (skip && *skip) return;
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < R;
       r += (uint64_t)gridDim.x * blockDim.x)
    analytic_one(kind, n, A, b, c, s1, theta, tau, u, Aa, NH, h, r, f);
}

// 1/sigma^2 and 1/sigma^4, formed once per thread: the kernel factors and mixture densities
// multiply by them instead of dividing in the per-contribution loops
struct InvSigma {
  double is2, is4;
  __device__ __forceinline__ explicit InvSigma(double sigma) {
    is2 = 1.0 / (sigma * sigma);
    is4 = is2 * is2;
  }
};

__device__ __forceinline__ double z_grad(double sg) { return sqrt(2.0 / kPi) / sg; }
__device__ __forceinline__ double z_diag(double sg) {
  return 4.0 * exp(-0.5) / (sg * sg * sqrt(2.0 * kPi));
}

// per draw: F_s (antithetic pair collapsed, HVP difference quotient applied),
// divided by the aggregate mixture q(tau_s); v^T tau_s for the limit HVP
__device__ __forceinline__ void prep_one(const EstShape& e, const double* __restrict__ f,
                                         const double* __restrict__ tau,
                                         const double* __restrict__ vnorm,
                                         const double* __restrict__ v, uint64_t sidx,
                                         double* __restrict__ Fq, double* __restrict__ vt) {
  {
    const uint64_t r0 = sidx * (uint64_t)(e.A * e.NH);
    double F0, F1 = 0.0;
    if (e.what == kHvp && e.pair) {
      // the loss differences f(+h) - f(-h) of the draw's pairs
      const double vn = *vnorm;
      const uint64_t p0 = sidx * (uint64_t)e.A;
      F0 = vn * f[p0] / (2.0 * e.h);
      if (e.A == 2) F1 = vn * f[p0 + 1] / (2.0 * e.h);
    } else if (e.what == kHvp) {
      const double vn = *vnorm;
      F0 = vn * (f[r0 + 0] - f[r0 + 1]) / (2.0 * e.h);
      if (e.A == 2) F1 = vn * (f[r0 + 2] - f[r0 + 3]) / (2.0 * e.h);
    } else {
      F0 = f[r0];
      if (e.A == 2) F1 = f[r0 + 1];
    }
    double F = F0;
    // even weights (Hessian kernel, plain loss) add the antithetic partner
    if (e.A == 2) F = (e.hessk || e.what == kLoss) ? F0 + F1 : F0 - F1;
    const double* t = tau + sidx * (uint64_t)e.n;
    const double sg = e.sigma;
    const InvSigma iv(sg);
    if (e.sampler == kAIS) {
      double q = 0.0;
      if (!e.hessk) {
        // q = 1/K sum_k |d_k| / Z_G with |d_k| = |t_k| / sigma^2
        const double c = iv.is2 / z_grad(sg);
        // loads eight ahead of the (ordered) additions
        int k = 0;
        for (; k + 8 <= e.n; k += 8) {
          double tk[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) tk[u] = t[k + u];
#pragma unroll
          for (int u = 0; u < 8; ++u) q += fabs(tk[u]) * c;
        }
        for (; k < e.n; ++k) q += fabs(t[k]) * c;
      } else {
        const double izd = 1.0 / z_diag(sg), izo = 1.0 / (z_grad(sg) * z_grad(sg));
        double l1 = 0.0, l2 = 0.0, qd = 0.0;
        auto add = [&](double tk) {
          qd += fabs(tk * tk * iv.is4 - iv.is2) * izd;
          l1 += fabs(tk);
          l2 += tk * tk;
        };
        int k = 0;
        for (; k + 8 <= e.n; k += 8) {
          double tk[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) tk[u] = t[k + u];
#pragma unroll
          for (int u = 0; u < 8; ++u) add(tk[u]);
        }
        for (; k < e.n; ++k) add(t[k]);
        // sum_{i<j} |t_i t_j| = ((sum |t_i|)^2 - sum t_i^2) / 2; the n^2 mixture
        // counts each off-diagonal pair twice and divides by n^2
        const double off = 0.5 * (l1 * l1 - l2) * iv.is4 * izo;
        q = e.mix_n2 ? qd + 2.0 * off : qd + off;
      }
      q /= e.mix_n2 ? (double)e.n * (double)e.n : (double)e.K;
      F /= q;
    }
    Fq[sidx] = F;
    if (e.what == kHvpLimit) {
      double acc = 0.0;
      for (int k = 0; k < e.n; ++k) acc += v[k] * t[k];
      vt[sidx] = acc;
    }
  }
}

__global__ void k_prep(EstShape e, const double* __restrict__ f, const double* __restrict__ tau,
                       const double* __restrict__ vnorm, const double* __restrict__ v,
                       double* __restrict__ Fq, double* __restrict__ vt) {
  if (e.skip && *e.skip) return;
  const uint64_t total = e.streams * e.N;
  for (uint64_t sidx = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; sidx < total;
       sidx += (uint64_t)gridDim.x * blockDim.x)
    prep_one(e, f, tau, vnorm, v, sidx, Fq, vt);
}

// kernel factor d_m(tau) (output m; Hessian elements from (i, j))
__device__ __forceinline__ double kfac(const EstShape& e, const InvSigma& iv, int m, int i, int j,
                                       const double* t, double vts, const double* v) {
  if (e.what == kLoss) return 1.0;   // smoothed loss: plain mean of the renders
  if (e.what == kHvpLimit) return t[m] * vts * iv.is4 - v[m] * iv.is2;
  if (!e.hessk) return -t[m] * iv.is2;
  if (i == j) return t[i] * t[i] * iv.is4 - iv.is2;
  return t[i] * t[j] * iv.is4;
}

struct Lobes32 { fsum2 pos, neg; };

// aggregate / Gaussian / limit HVP: block = chunk of draws, threads = elements
constexpr int kLdsDoubles = 3072;   // 24 KiB of draws per chunk (six blocks per CU)
static_assert(kLdsDoubles >= kMaxParams, "a chunk holds at least one draw of every scene");

struct AccumLds {
  double tau[kLdsDoubles];
  double F[256];
  double vt[256];
};

__device__ __forceinline__ void accum_block(const EstShape& e, const double* __restrict__ tau,
                                            const double* __restrict__ Fq,
                                            const double* __restrict__ vt,
                                            const double* __restrict__ v, int fp64, int chunk,
                                            uint64_t c, void* __restrict__ part, AccumLds& L_) {
  double* s_tau = L_.tau;
  double* s_F = L_.F;
  double* s_vt = L_.vt;
  __syncthreads();   // the previous task's readers of LDS are done
  const uint64_t s0 = c * (uint64_t)chunk;
  const int ns = (int)min((uint64_t)chunk, e.N - s0);
  {
    // eight loads in flight per thread before their LDS stores (a plain loop
    // waits for every load before the next one is issued)
    const double* __restrict__ src = tau + s0 * (uint64_t)e.n;
    const int tot = ns * e.n, st = (int)blockDim.x;
    int i = threadIdx.x;
    for (; i + 7 * st < tot; i += 8 * st) {
      double r[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) r[u] = src[i + u * st];
#pragma unroll
      for (int u = 0; u < 8; ++u) s_tau[i + u * st] = r[u];
    }
    for (; i < tot; i += st) s_tau[i] = src[i];
  }
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    s_F[i] = Fq[s0 + i];
    s_vt[i] = e.what == kHvpLimit ? vt[s0 + i] : 0.0;
  }
  __syncthreads();
  const InvSigma iv(e.sigma);
  for (int m = threadIdx.x; m < e.nout; m += blockDim.x) {
    int i = 0, j = 0;
    if (e.hessk && e.what == kHess) tri_ij(e.n, m, i, j);
    if (fp64) {
      double pos = 0.0, neg = 0.0;
      for (int s = 0; s < ns; ++s) {
        const double cv = kfac(e, iv, m, i, j, s_tau + s * e.n, s_vt[s], v) * s_F[s];
        if (cv >= 0.0) pos += cv; else neg -= cv;
      }
      ((double2*)part)[c * (uint64_t)e.nout + m] = make_double2(pos, neg);
    } else {
      Lobes32 L = {{0.f, 0.f}, {0.f, 0.f}};
      for (int s = 0; s < ns; ++s) {
        const float cv = (float)(kfac(e, iv, m, i, j, s_tau + s * e.n, s_vt[s], v) * s_F[s]);
        if (cv >= 0.0f) two_sum_add(L.pos, cv); else two_sum_add(L.neg, -cv);
      }
      ((float4*)part)[c * (uint64_t)e.nout + m] = make_float4(L.pos.hi, L.pos.lo, L.neg.hi, L.neg.lo);
    }
  }
}

__global__ __launch_bounds__(256) void k_accum(EstShape e, const double* __restrict__ tau,
                                               const double* __restrict__ Fq,
                                               const double* __restrict__ vt,
                                               const double* __restrict__ v, int fp64,
                                               int chunk, void* __restrict__ part) {
  __shared__ AccumLds lds;
  if (e.skip && *e.skip) return;
  accum_block(e, tau, Fq, vt, v, fp64, chunk, blockIdx.x, part, lds);
}

// per-element IS: (element, chunk) item gid, draws of that element's stream
__device__ __forceinline__ void accum_is_one(const EstShape& e, const double* __restrict__ tau,
                                             const double* __restrict__ Fq, int fp64, int chunk,
                                             uint64_t gid, void* __restrict__ part) {
  const int m = (int)(gid % (uint64_t)e.nout);
  const uint64_t c = gid / (uint64_t)e.nout;
  const uint64_t s0 = c * (uint64_t)chunk;
  const int ns = (int)min((uint64_t)chunk, e.N - s0);
  int i = m, j = m;
  if (e.hessk) tri_ij(e.n, m, i, j);
  const InvSigma iv(e.sigma);
  const double zm = !e.hessk ? z_grad(e.sigma) : (i == j ? z_diag(e.sigma) : z_grad(e.sigma) * z_grad(e.sigma));
  double pos64 = 0.0, neg64 = 0.0;
  Lobes32 L = {{0.f, 0.f}, {0.f, 0.f}};
  for (int s = 0; s < ns; ++s) {
    const uint64_t sidx = (uint64_t)m * e.N + s0 + s;
    const double* t = tau + sidx * (uint64_t)e.n;
    const double d = kfac(e, iv, m, i, j, t, 0.0, nullptr);
    const double w = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) * zm;
    const double cv = w * Fq[sidx];
    if (fp64) {
      if (cv >= 0.0) pos64 += cv; else neg64 -= cv;
    } else {
      const float cf = (float)cv;
      if (cf >= 0.0f) two_sum_add(L.pos, cf); else two_sum_add(L.neg, -cf);
    }
  }
  if (fp64) ((double2*)part)[c * (uint64_t)e.nout + m] = make_double2(pos64, neg64);
  else ((float4*)part)[c * (uint64_t)e.nout + m] = make_float4(L.pos.hi, L.pos.lo, L.neg.hi, L.neg.lo);
}

__global__ void k_accum_is(EstShape e, const double* __restrict__ tau,
                           const double* __restrict__ Fq, int fp64, int chunk, uint64_t nchunks,
                           void* __restrict__ part) {
  if (e.skip && *e.skip) return;
  const uint64_t total = nchunks * (uint64_t)e.nout;
  for (uint64_t gid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; gid < total;
       gid += (uint64_t)gridDim.x * blockDim.x)
    accum_is_one(e, tau, Fq, fp64, chunk, gid, part);
}

// FP64 lobe difference over chunks in fixed order; Hessian mirrored.
// One block per element: thread t sums chunks t, t + 256, ... and the 256
// partial sums meet in a fixed pairing tree.
__device__ __forceinline__ void finalize_block(const EstShape& e, const void* __restrict__ part,
                                               int fp64, uint64_t nchunks, int m,
                                               double* __restrict__ out, double* s_pos,
                                               double* s_neg) {
  __syncthreads();   // the previous task's readers of LDS are done
  double pos = 0.0, neg = 0.0;
  for (uint64_t c = threadIdx.x; c < nchunks; c += blockDim.x) {
    if (fp64) {
      const double2 p = ((const double2*)part)[c * (uint64_t)e.nout + m];
      pos += p.x;
      neg += p.y;
    } else {
      const float4 p = ((const float4*)part)[c * (uint64_t)e.nout + m];
      pos += (double)p.x + (double)p.y;
      neg += (double)p.z + (double)p.w;
    }
  }
  s_pos[threadIdx.x] = pos;
  s_neg[threadIdx.x] = neg;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_pos[threadIdx.x] += s_pos[threadIdx.x + off];
      s_neg[threadIdx.x] += s_neg[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double est = (s_pos[0] - s_neg[0]) / ((double)e.A * (double)e.N);
  if (e.what == kHess) {
    int i, j;
    tri_ij(e.n, m, i, j);
    out[i * e.n + j] = est;
    out[j * e.n + i] = est;
  } else {
    out[m] = est;
  }
}

__global__ __launch_bounds__(256) void k_finalize(EstShape e, const void* __restrict__ part,
                                                  int fp64, uint64_t nchunks,
                                                  double* __restrict__ out) {
  __shared__ double s_pos[256], s_neg[256];
  if (e.skip && *e.skip) return;
  finalize_block(e, part, fp64, nchunks, blockIdx.x, out, s_pos, s_neg);
}

// ---- batch phase kernels: the same bodies over the task lists ----
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// elements [t * kElems, min(total, (t + 1) * kElems)) of a step
template <int kElems = kBatchElems, class F>
__device__ __forceinline__ void elems_of_task(uint64_t t, uint64_t total, F&& fn) {
  const uint64_t b = t * (uint64_t)kElems;
  const uint64_t e = umin64(total, b + kElems);
  for (uint64_t g = b + threadIdx.x; g < e; g += blockDim.x) fn(g);
}

__global__ __launch_bounds__(256) void k_batch_sample(const BatchTable* __restrict__ T) {
  __shared__ double s_acc[256];
  const int nq = T->nq;
  const uint64_t* off = T->off + (uint64_t)kPhSample * (nq + 1);
  // the render work queues start empty
  if (blockIdx.x == 0 && threadIdx.x < kWorkCounters) T->ctr[threadIdx.x] = 0ull;
  const uint64_t total = off[nq];
  for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = batch_find(off, nq, t);
    const BatchQuery& Q = T->q[q];
    uint64_t lt = t - off[q];
    const bool hv = Q.e.what == kHvp || Q.e.what == kHvpLimit;
    if (hv) {
      if (lt == 0) {
        vnorm_block(Q.e.n, Q.v, Q.u, Q.u + Q.e.n, s_acc);
        continue;
      }
      lt -= 1;
    }
    const EstShape& e = Q.e;
    elems_of_task(lt, e.streams * e.N * (uint64_t)e.n, [&](uint64_t g) {
      sample_one(e.n, e.K, e.hessk, e.mix_n2, e.sampler, e.N, e.seed, e.sigma, g, Q.tau);
    });
  }
}

__global__ __launch_bounds__(256) void k_batch_analytic(const BatchTable* __restrict__ T) {
  const int nq = T->nq;
  const uint64_t* off = T->off + (uint64_t)kPhAnalytic * (nq + 1);
  const uint64_t total = off[nq];
  for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = batch_find(off, nq, t);
    const BatchQuery& Q = T->q[q];
    const EstShape& e = Q.e;
    const AnalyticScene& a = Q.as;
    elems_of_task<kBatchHeavyElems>(t - off[q], e.R, [&](uint64_t r) {
      analytic_one(a.kind, a.n, a.A, a.b, a.c, a.s1, Q.theta, Q.tau, Q.u, e.A, e.NH, e.h, r, Q.f);
    });
  }
}

__global__ __launch_bounds__(256) void k_batch_prep(const BatchTable* __restrict__ T) {
  const int nq = T->nq;
  const uint64_t* off = T->off + (uint64_t)kPhPrep * (nq + 1);
  const uint64_t total = off[nq];
  for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = batch_find(off, nq, t);
    const BatchQuery& Q = T->q[q];
    elems_of_task<kBatchHeavyElems>(t - off[q], Q.e.streams * Q.e.N, [&](uint64_t sidx) {
      prep_one(Q.e, Q.f, Q.tau, Q.u + Q.e.n, Q.v, sidx, Q.Fq, Q.vt);
    });
  }
}

__global__ __launch_bounds__(256) void k_batch_accum(const BatchTable* __restrict__ T) {
  __shared__ AccumLds lds;
  const int nq = T->nq;
  const uint64_t* off = T->off + (uint64_t)kPhAccum * (nq + 1);
  const uint64_t total = off[nq];
  for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = batch_find(off, nq, t);
    const BatchQuery& Q = T->q[q];
    const uint64_t lt = t - off[q];
    if (per_element(Q.e.sampler)) {
      // 256 (element, chunk) items per task, as 256-thread blocks
      const uint64_t g = lt * 256u + threadIdx.x;
      if (g < Q.nchunks * (uint64_t)Q.e.nout) accum_is_one(Q.e, Q.tau, Q.Fq, Q.fp64, Q.chunk, g, Q.acc);
    } else {
      accum_block(Q.e, Q.tau, Q.Fq, Q.vt, Q.v, Q.fp64, Q.chunk, lt, Q.acc, lds);
    }
  }
}

__global__ __launch_bounds__(256) void k_batch_finalize(const BatchTable* __restrict__ T) {
  __shared__ double s_pos[256], s_neg[256];
  const int nq = T->nq;
  const uint64_t* off = T->off + (uint64_t)kPhFinalize * (nq + 1);
  const uint64_t total = off[nq];
  for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = batch_find(off, nq, t);
    const BatchQuery& Q = T->q[q];
    finalize_block(Q.e, Q.acc, Q.fp64, Q.nchunks, (int)(t - off[q]), Q.out, s_pos, s_neg);
  }
}

}  // namespace

void launch_sample(hipStream_t st, const EstShape& e, double* tau) {
  const uint64_t total = e.streams * e.N * (uint64_t)e.n;
  hipLaunchKernelGGL(k_sample, dim3(grid_for(total, 256)), dim3(256), 0, st, e.n, e.K, e.hessk,
                     e.mix_n2, e.sampler, e.N, e.seed, e.sigma, total, tau, e.skip);
}

void launch_sample_vnorm(hipStream_t st, const EstShape& e, double* tau, const double* v,
                         double* u, double* vnorm, bool draws) {
  const uint64_t total = draws ? e.streams * e.N * (uint64_t)e.n : 0;
  hipLaunchKernelGGL(k_sample_vnorm, dim3(grid_for(total, 256)), dim3(256), 0, st, e.n, e.K,
                     e.hessk, e.mix_n2, e.sampler, e.N, e.seed, e.sigma, total, tau, v, u, vnorm,
                     e.skip);
}


void launch_analytic(hipStream_t st, const EstShape& e, const AnalyticScene& s,
                     const double* theta, const double* tau, const double* u, double* f) {
  hipLaunchKernelGGL(k_analytic, dim3(grid_for(e.R, 128)), dim3(128), 0, st, s.kind, s.n, s.A, s.b,
                     s.c, s.s1, theta, tau, u, e.A, e.NH, e.h, e.R, f, e.skip);
}

void launch_prep(hipStream_t st, const EstShape& e, const double* f, const double* tau,
                 const double* vnorm, const double* v, double* Fq, double* vt) {
  hipLaunchKernelGGL(k_prep, dim3(grid_for(e.streams * e.N, 128)), dim3(128), 0, st, e, f, tau,
                     vnorm, v, Fq, vt);
}

// Draws per accumulation chunk: as many as LDS holds (at most 256), but for
// few outputs (a block's threads are its outputs, each summing its chunk's
// draws in one dependent chain) no more than max(16, N / 512), so that short
// chains over many blocks replace long chains over a few.
int accum_chunk(const EstShape& e) {
  if (per_element(e.sampler)) return 256;
  int c = kLdsDoubles / e.n;
  if (c > 256) c = 256;
  const uint64_t lim = e.N / 512 > 16 ? e.N / 512 : 16;
  if ((uint64_t)c > lim) c = (int)lim;
  if (c < 1) c = 1;
  return c;
}

void launch_accum(hipStream_t st, const EstShape& e, const double* tau, const double* Fq,
                  const double* vt, const double* v, int fp64, void* part, int chunk) {
  const uint64_t nchunks = (e.N + chunk - 1) / chunk;
  if (per_element(e.sampler)) {
    hipLaunchKernelGGL(k_accum_is, dim3(grid_for(nchunks * e.nout, 128)), dim3(128), 0, st, e, tau,
                       Fq, fp64, chunk, nchunks, part);
  } else {
    hipLaunchKernelGGL(k_accum, dim3((unsigned)nchunks), dim3(256), 0, st, e, tau, Fq, vt, v, fp64,
                       chunk, part);
  }
}

void launch_finalize(hipStream_t st, const EstShape& e, const void* part, int fp64, int chunk,
                     double* out) {
  const uint64_t nchunks = (e.N + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)e.nout), dim3(256), 0, st, e, part, fp64, nchunks,
                     out);
}

uint64_t batch_tasks(const BatchQuery& q, int phase) {
  const EstShape& e = q.e;
  auto ceil_div = [](uint64_t a, uint64_t b) { return (a + b - 1) / b; };
  const bool render = q.scene == kDisks || q.scene == kPT;
  switch (phase) {
    case kPhSample:
      return ((e.what == kHvp || e.what == kHvpLimit) ? 1 : 0) +
             ceil_div(e.streams * e.N * (uint64_t)e.n, kBatchElems);
    case kPhRecords:   // render pairs build their records in the raster kernel
      return q.scene == kDisks && !e.pair ? ceil_div(e.R * (uint64_t)q.ds.D, kBatchElems) : 0;
    case kPhAnalytic:
      return render ? 0 : ceil_div(e.R, kBatchHeavyElems);
    case kPhReduce:    // and write their loss differences directly
      return render && !(q.scene == kDisks && e.pair) ? ceil_div(e.R, kBatchRenders) : 0;
    case kPhPrep:
      return ceil_div(e.streams * e.N, kBatchHeavyElems);
    case kPhAccum:
      return per_element(e.sampler) ? ceil_div(q.nchunks * (uint64_t)e.nout, 256) : q.nchunks;
    case kPhFinalize:
      return (uint64_t)e.nout;
    default:
      return 0;
  }
}

void launch_batch_sample(hipStream_t st, const BatchTable* T, int blocks) {
  hipLaunchKernelGGL(k_batch_sample, dim3(blocks), dim3(256), 0, st, T);
}
void launch_batch_analytic(hipStream_t st, const BatchTable* T, int blocks) {
  hipLaunchKernelGGL(k_batch_analytic, dim3(blocks), dim3(256), 0, st, T);
}
void launch_batch_prep(hipStream_t st, const BatchTable* T, int blocks) {
  hipLaunchKernelGGL(k_batch_prep, dim3(blocks), dim3(256), 0, st, T);
}
void launch_batch_accum(hipStream_t st, const BatchTable* T, int blocks) {
  hipLaunchKernelGGL(k_batch_accum, dim3(blocks), dim3(256), 0, st, T);
}
void launch_batch_finalize(hipStream_t st, const BatchTable* T, int blocks) {
  hipLaunchKernelGGL(k_batch_finalize, dim3(blocks), dim3(256), 0, st, T);
}

}  // namespace hr
