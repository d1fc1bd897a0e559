// hr_solve.hip -- FP64 solver steps on the GPU (single work-group kernels).
//
// Newton-CG (section "Previous Work" of Wang, Fischer, Ritschel 2025):
//   v0 = r0 = -g;  alpha = r^T r / v^T H v  (= -g^T v / v^T H v on the first step);
//   alpha <- min(alpha, Delta / |v|) (trust truncation, ends the inner loop);
//   v^T H v <= 0 -> move to the trust boundary along v and stop;
//   r <- r - alpha H v;  beta = r_new^T r_new / r^T r (Fletcher-Reeves);  v <- r + beta v.
// With `modified` set the exits are replaced by the paper's Hessian
// modification: the curvature becomes max(|v^T H v|, floor |v|^2), the step is
// truncated to Delta/|v| and CG continues for all its iterations.
// Modified Newton on a full estimate (appendix on non-PSD Hessians): cyclic
// Jacobi eigen-decomposition, |lambda| floored, step scaled into Delta.
#include "hr_kernels.h"

namespace hr {

namespace {

constexpr int kThreads = 256;

// deterministic block sum (fixed pairing tree)
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = kThreads / 2; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kThreads) void k_cg_init(int n, const double* __restrict__ g,
                                                      double delta, int modified,
                                                      double eig_floor, double* r, double* p,
                                                      double* d, CgState* cs) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    r[i] = -g[i];
    p[i] = -g[i];
    d[i] = 0.0;
    acc += g[i] * g[i];
  }
  const double gg = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    cs->rr = gg;
    cs->gnorm = sqrt(gg);
    cs->delta = delta;
    cs->iters = 0;
    cs->hit_trust = 0;
    cs->neg_curv = 0;
    cs->step_norm = 0.0;
    cs->modified = modified;
    cs->eig_floor = eig_floor;
    cs->stop = gg == 0.0 ? 1 : 0;
  }
}

__global__ __launch_bounds__(kThreads) void k_cg_update(int n, const double* __restrict__ Hp,
                                                        double* r, double* p, double* d,
                                                        CgState* cs) {
  __shared__ double sh[kThreads];
  __shared__ int s_mode;
  __shared__ double s_alpha;
  if (cs->stop) return;   // uniform: every thread reads the same flag
  double a1 = 0.0, a2 = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    a1 += p[i] * Hp[i];
    a2 += p[i] * p[i];
  }
  const double curv = block_sum(a1, sh);
  const double pn = sqrt(block_sum(a2, sh));
  if (threadIdx.x == 0) {
    cs->iters += 1;
    if (pn == 0.0) {
      s_mode = 3;
      s_alpha = 0.0;
    } else if (cs->modified) {
      // Hessian modification inside CG: |curvature|, floored; truncated
      // steps continue
      double kappa = fabs(curv);
      if (curv <= 0.0) cs->neg_curv = 1;
      const double fl = cs->eig_floor * pn * pn;
      if (kappa < fl) kappa = fl;
      if (kappa == 0.0) {
        s_mode = 3;
        s_alpha = 0.0;
      } else {
        double alpha = cs->rr / kappa;
        if (alpha > cs->delta / pn) {
          alpha = cs->delta / pn;
          cs->hit_trust = 1;
        }
        s_mode = 0;
        s_alpha = alpha;
      }
    } else if (curv <= 0.0) {
      s_mode = 1;
      s_alpha = cs->delta / pn;
      cs->neg_curv = 1;
    } else {
      double alpha = cs->rr / curv;
      if (alpha > cs->delta / pn) {
        s_mode = 2;
        s_alpha = cs->delta / pn;
        cs->hit_trust = 1;
      } else {
        s_mode = 0;
        s_alpha = alpha;
      }
    }
  }
  __syncthreads();
  const int mode = s_mode;
  const double alpha = s_alpha;
  for (int i = threadIdx.x; i < n; i += kThreads) d[i] += alpha * p[i];
  if (mode != 0) {
    if (threadIdx.x == 0) cs->stop = 1;
    return;
  }
  double a3 = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    r[i] -= alpha * Hp[i];
    a3 += r[i] * r[i];
  }
  const double rr_new = block_sum(a3, sh);
  const double rr_old = cs->rr;
  const bool done = sqrt(rr_new) <= 1e-10 * cs->gnorm;
  const double beta = rr_new / rr_old;
  if (!done)
    for (int i = threadIdx.x; i < n; i += kThreads) p[i] = r[i] + beta * p[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    cs->rr = rr_new;
    if (done) cs->stop = 1;
  }
}

__global__ __launch_bounds__(kThreads) void k_cg_apply(int n, const double* __restrict__ d,
                                                       double* theta, CgState* cs) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    theta[i] += d[i];
    acc += d[i] * d[i];
  }
  const double dd = block_sum(acc, sh);
  if (threadIdx.x == 0) cs->step_norm = sqrt(dd);
}

// modified Newton: work = [A (n*n) | V (n*n)]
__global__ __launch_bounds__(kThreads) void k_newton_full(int n, const double* __restrict__ H,
                                                          const double* __restrict__ g,
                                                          double delta, double eig_floor,
                                                          double* work, double* d, CgState* cs) {
  __shared__ double sh[kThreads];
  __shared__ double s_c, s_s;
  __shared__ int s_skip;
  double* A = work;
  double* V = work + (size_t)n * n;
  for (int i = threadIdx.x; i < n * n; i += kThreads) {
    A[i] = H[i];
    V[i] = (i / n == i % n) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = threadIdx.x; i < n * n; i += kThreads) {
      const double a = A[i] * A[i];
      tot += a;
      if (i / n != i % n) off += a;
    }
    off = block_sum(off, sh);
    tot = block_sum(tot, sh);
    if (off == 0.0 || off <= 1e-30 * tot) break;
    for (int pp = 0; pp < n - 1; ++pp) {
      for (int q = pp + 1; q < n; ++q) {
        if (threadIdx.x == 0) {
          const double apq = A[pp * n + q];
          s_skip = apq == 0.0;
          if (!s_skip) {
            const double th = (A[q * n + q] - A[pp * n + pp]) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            s_c = 1.0 / sqrt(t * t + 1.0);
            s_s = t * s_c;
          }
        }
        __syncthreads();
        if (!s_skip) {
          const double c = s_c, s = s_s;
          for (int k = threadIdx.x; k < n; k += kThreads) {
            const double akp = A[k * n + pp], akq = A[k * n + q];
            A[k * n + pp] = c * akp - s * akq;
            A[k * n + q] = s * akp + c * akq;
          }
          __syncthreads();
          for (int k = threadIdx.x; k < n; k += kThreads) {
            const double apk = A[pp * n + k], aqk = A[q * n + k];
            A[pp * n + k] = c * apk - s * aqk;
            A[q * n + k] = s * apk + c * aqk;
            const double vkp = V[k * n + pp], vkq = V[k * n + q];
            V[k * n + pp] = c * vkp - s * vkq;
            V[k * n + q] = s * vkp + c * vkq;
          }
        }
        __syncthreads();
      }
    }
  }
  // d = -sum_k V_k (V_k^T g) / max(|lambda_k|, floor)
  for (int i = threadIdx.x; i < n; i += kThreads) d[i] = 0.0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    double lam = fabs(A[k * n + k]);
    if (lam < eig_floor) lam = eig_floor;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) acc += V[i * n + k] * g[i];
    const double proj = block_sum(acc, sh);
    if (lam == 0.0) continue;
    for (int i = threadIdx.x; i < n; i += kThreads) d[i] -= V[i * n + k] * proj / lam;
    __syncthreads();
  }
  double acc = 0.0, gg = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    acc += d[i] * d[i];
    gg += g[i] * g[i];
  }
  const double dn = sqrt(block_sum(acc, sh));
  const double gn = sqrt(block_sum(gg, sh));
  const bool clip = dn > delta;
  if (clip)
    for (int i = threadIdx.x; i < n; i += kThreads) d[i] *= delta / dn;
  if (threadIdx.x == 0) {
    cs->iters = 1;
    cs->hit_trust = clip ? 1 : 0;
    cs->neg_curv = 0;
    cs->gnorm = gn;
    cs->stop = 1;
    cs->delta = delta;
  }
}

// grey-box composition (appendix "Grey-box differentials"): small FP64
// contractions with the inner Jacobian, one thread per output element, sums
// in index order
__global__ void k_jt_vec(int n, int n_in, const double* __restrict__ J, const double* __restrict__ a,
                         double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_in) return;
  double acc = 0.0;
  for (int i = 0; i < n; ++i) acc += J[(size_t)i * n_in + c] * a[i];
  out[c] = acc;
}

__global__ void k_j_vec(int n, int n_in, const double* __restrict__ J, const double* __restrict__ v,
                        double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int c = 0; c < n_in; ++c) acc += J[(size_t)i * n_in + c] * v[c];
  out[i] = acc;
}

// T = H J (n x n_in)
__global__ void k_h_j(int n, int n_in, const double* __restrict__ J, const double* __restrict__ H,
                      double* __restrict__ T) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n_in) return;
  const int i = (int)(e / n_in), c = (int)(e % n_in);
  double acc = 0.0;
  for (int k = 0; k < n; ++k) acc += H[(size_t)i * n + k] * J[(size_t)k * n_in + c];
  T[e] = acc;
}

// out = J^T T (n_in x n_in)
__global__ void k_jt_t(int n, int n_in, const double* __restrict__ J, const double* __restrict__ T,
                       double* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n_in * n_in) return;
  const int a = (int)(e / n_in), b = (int)(e % n_in);
  double acc = 0.0;
  for (int i = 0; i < n; ++i) acc += J[(size_t)i * n_in + a] * T[(size_t)i * n_in + b];
  out[e] = acc;
}

}  // namespace

void launch_jt_vec(hipStream_t st, int n, int n_in, const double* J, const double* a, double* out) {
  hipLaunchKernelGGL(k_jt_vec, dim3((n_in + 127) / 128), dim3(128), 0, st, n, n_in, J, a, out);
}
void launch_j_vec(hipStream_t st, int n, int n_in, const double* J, const double* v, double* out) {
  hipLaunchKernelGGL(k_j_vec, dim3((n + 127) / 128), dim3(128), 0, st, n, n_in, J, v, out);
}
void launch_jt_h_j(hipStream_t st, int n, int n_in, const double* J, const double* H, double* T,
                   double* out) {
  const size_t e1 = (size_t)n * n_in, e2 = (size_t)n_in * n_in;
  hipLaunchKernelGGL(k_h_j, dim3((unsigned)((e1 + 127) / 128)), dim3(128), 0, st, n, n_in, J, H, T);
  hipLaunchKernelGGL(k_jt_t, dim3((unsigned)((e2 + 127) / 128)), dim3(128), 0, st, n, n_in, J, T,
                     out);
}

void launch_cg_init(hipStream_t st, int n, const double* g, double delta, int modified,
                    double eig_floor, double* r, double* p, double* d, CgState* cs) {
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(kThreads), 0, st, n, g, delta, modified, eig_floor,
                     r, p, d, cs);
}
void launch_cg_update(hipStream_t st, int n, const double* Hp, double* r, double* p, double* d,
                      CgState* cs) {
  hipLaunchKernelGGL(k_cg_update, dim3(1), dim3(kThreads), 0, st, n, Hp, r, p, d, cs);
}
void launch_cg_apply(hipStream_t st, int n, const double* d, double* theta, CgState* cs) {
  hipLaunchKernelGGL(k_cg_apply, dim3(1), dim3(kThreads), 0, st, n, d, theta, cs);
}
void launch_newton_full(hipStream_t st, int n, const double* H, const double* g, double delta,
                        double eig_floor, double* work, double* d, CgState* cs) {
  hipLaunchKernelGGL(k_newton_full, dim3(1), dim3(kThreads), 0, st, n, H, g, delta, eig_floor,
                     work, d, cs);
}

}  // namespace hr
