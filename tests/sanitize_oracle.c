/*
 * Drives every entry point of the oracle on small scenes, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).
 * The values are not checked here (the oracle's pins do that); the run must
 * finish without a sanitizer report and without a leak.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "orc.h"

static int fails = 0;
#define CHECK(x)                                                    \
  do {                                                              \
    int rc_ = (x);                                                  \
    if (rc_ != 0) {                                                 \
      fprintf(stderr, "%s:%d: %s returned %d\n", __FILE__, __LINE__, #x, rc_); \
      ++fails;                                                      \
    }                                                               \
  } while (0)

static orc_opts opts(int sampler, int threads, double* dbg) {
  orc_opts o;
  memset(&o, 0, sizeof o);
  o.sampler = sampler;
  o.antithetic = 1;
  o.hvp_rel_step = 0.1;
  o.nthreads = threads;
  o.dbg_loss = dbg;
  return o;
}

/* gradient, Hessian, both HVPs and the smoothed loss with every sampler that
 * supports them; n parameters */
static void estimators(const orc_scene* sc, const double* th, int n, double sigma, int N) {
  double* out = (double*)calloc((size_t)n * n, sizeof(double));
  double* v = (double*)malloc((size_t)n * sizeof(double));
  double* dbg = (double*)calloc((size_t)N * n * 8, sizeof(double));
  for (int i = 0; i < n; ++i) v[i] = 1.0 - 0.3 * i;
  const int samplers[4] = {ORC_AIS, ORC_IS, ORC_GAUSS, ORC_FR22};
  for (int k = 0; k < 4; ++k) {
    const int sp = samplers[k];
    orc_opts o = opts(sp, k % 2 ? 2 : 1, k == 0 ? dbg : NULL);
    CHECK(orc_est_grad(sc, th, sigma, N, 3, &o, out));
    CHECK(orc_est_hvp(sc, th, sigma, N, 3, v, &o, out));
    if (sp != ORC_FR22) CHECK(orc_est_hessian(sc, th, sigma, N, 3, &o, out));
    if (sp == ORC_AIS || sp == ORC_GAUSS) CHECK(orc_est_hvp_limit(sc, th, sigma, N, 3, v, &o, out));
    if (sp == ORC_AIS) {
      o.hess_mix_n2 = 1;
      CHECK(orc_est_hessian(sc, th, sigma, N, 3, &o, out));
      o.hess_mix_n2 = 0;
      o.s0 = 5;
      CHECK(orc_est_grad(sc, th, sigma, N, 3, &o, out));
    }
  }
  orc_opts o = opts(ORC_AIS, 1, NULL);
  double F;
  CHECK(orc_est_loss(sc, th, sigma, N, 3, &o, &F));
  CHECK(orc_est_loss(sc, th, 0.0, 1, 3, &o, &F));
  free(out);
  free(v);
  free(dbg);
}

static void solvers(const orc_scene* sc, const double* th0, int n, double sigma, int N) {
  double* th = (double*)malloc((size_t)n * sizeof(double));
  orc_opts o = opts(ORC_AIS, 2, NULL);
  orc_ncg_opts no;
  memset(&no, 0, sizeof no);
  no.cg_iters = 3;
  no.trust_radius = 0.05;
  no.eig_floor = 1e-3;
  orc_ncg_report rep;
  for (int mode = 0; mode < 4; ++mode) {
    memcpy(th, th0, (size_t)n * sizeof(double));
    no.use_full_hessian = mode == 1;
    no.hvp_limit = mode == 2;
    no.modified = mode == 3;
    CHECK(orc_newton_cg_step(sc, th, sigma, N, 7, &no, &o, &rep));
  }
  orc_optim_opts oo;
  memset(&oo, 0, sizeof oo);
  oo.iters = 2;
  oo.sigma_start = sigma;
  oo.sigma_end = 0.5 * sigma;
  oo.lr = 0.1;
  oo.ls_iters = 2;
  oo.ls_tol = 1e-4;
  oo.recompute = 1;
  oo.N_loss = 8;
  oo.ncg = no;
  double trace[2 * 5];
  for (int m = 0; m < 3; ++m) {
    memcpy(th, th0, (size_t)n * sizeof(double));
    oo.method = m;
    CHECK(orc_optimize(sc, th, N, 9, &oo, &o, trace));
  }
  free(th);
}

static void greybox(const orc_scene* sc, const double* y, int n, double sigma, int N) {
  const int n_in = 2;
  double* J = (double*)malloc((size_t)n * n_in * sizeof(double));
  for (int i = 0; i < n * n_in; ++i) J[i] = 0.1 * (i % 5) - 0.2;
  double out[4], vx[2] = {1.0, -0.5};
  orc_opts o = opts(ORC_AIS, 1, NULL);
  CHECK(orc_est_grad_greybox(sc, y, J, n_in, sigma, N, 3, &o, out));
  CHECK(orc_est_hessian_greybox(sc, y, J, n_in, sigma, N, 3, &o, out));
  CHECK(orc_est_hvp_greybox(sc, y, J, n_in, sigma, N, 3, vx, &o, out));
  free(J);
}

int main(void) {
  /* random numbers and 1-D samplers */
  uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, w[4];
  orc_philox4x32_10(ctr, key, w);
  double acc = 0.0;
  const uint32_t words[6] = {0u, 1u, 0x7FFFFFFFu, 0x80000000u, 0xFFFFFFFEu, 0xFFFFFFFFu};
  for (int i = 0; i < 6; ++i)
    acc += orc_grad_lobe_icdf(words[i], 0.3) + orc_hdiag_icdf(words[i], 0.3);
  acc += orc_hdiag_cdf(0.1, 0.3) + orc_lambertw(-0.2, 0) + orc_lambertw(-0.2, -1);
  double tau[64];
  int el = 0;
  for (int sp = 0; sp < 3; ++sp)
    for (int what = 0; what < 2; ++what) CHECK(orc_draw_tau(what, 5, 0.2, 1, 2, sp, 0, 1, tau, &el));

  /* disks: RGB, (cx, cy, r) per disk, ragged 23 x 17 image, one disk with a
   * negative radius */
  {
    const int W = 23, H = 17, C = 3, D = 4, n = 3 * D;
    float colors[12], target[23 * 17 * 3];
    for (int i = 0; i < 12; ++i) colors[i] = 0.1f * (float)(i + 1);
    for (int i = 0; i < W * H * C; ++i) target[i] = (float)(i % 7) / 7.0f;
    orc_scene* sc = orc_scene_disks(W, H, C, D, 3, NULL, colors, target);
    const double th[12] = {0.3, 0.4, 0.2, 0.6, 0.5, 0.15, 0.5, 0.7, -0.01, 0.45, 0.45, 0.1};
    double* img = (double*)malloc((size_t)W * H * C * sizeof(double));
    CHECK(orc_render(sc, th, 0, 0, 0, img));
    acc += img[5] + orc_loss(sc, th, 0, 0);
    free(img);
    estimators(sc, th, n, 0.05, 12);
    solvers(sc, th, n, 0.05, 8);
    greybox(sc, th, n, 0.05, 8);
    orc_scene_free(sc);
  }
  /* disks with fixed radii, (cx, cy) per disk, one channel */
  {
    const int W = 16, H = 16, D = 2;
    const float radius[2] = {0.2f, 0.3f}, colors[2] = {1.0f, 0.5f};
    float target[256];
    for (int i = 0; i < 256; ++i) target[i] = 0.25f;
    orc_scene* sc = orc_scene_disks(W, H, 1, D, 2, radius, colors, target);
    const double th[4] = {0.4, 0.5, 0.6, 0.5};
    estimators(sc, th, 4, 0.05, 10);
    orc_scene_free(sc);
  }
  /* path tracer: two spheres on the plane, 6 x 5 pixels, 1 spp */
  {
    const double desc[26] = {0.0, 1.6, -3.5, 0.0, 0.3, 0.0, 45.0, 0.5, 8.0, 0.5, 0.5, 0.5,
                             0.2, 0.3, 0.1, 0.3, 0.6, 0.4, 0.3,
                             -0.5, 0.25, -0.2, 0.25, 0.3, 0.7, 0.5};
    float target[6 * 5 * 3];
    for (int i = 0; i < 90; ++i) target[i] = 0.1f;
    orc_scene* sc = orc_scene_pt(6, 5, 1, 2, desc, target);
    const double th[6] = {0.1, 2.0, 0.0, 0.2, 0.3, 0.1};
    double* img = (double*)malloc(90 * sizeof(double));
    CHECK(orc_render(sc, th, 4, 1, 2, img));
    free(img);
    const double o[3] = {0.0, 1.6, -3.5}, d[3] = {0.0, -0.3, 0.954};
    const double u[8] = {0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8};
    double t, L[3];
    (void)orc_pt_trace(sc, th, o, d, &t);
    CHECK(orc_pt_path(sc, th, o, d, u, L));
    orc_opts op = opts(ORC_AIS, 2, NULL);
    double g[6], Hm[36];
    CHECK(orc_est_grad(sc, th, 0.05, 4, 5, &op, g));
    CHECK(orc_est_hessian(sc, th, 0.05, 4, 5, &op, Hm));
    orc_scene_free(sc);
  }
  /* analytic scenes and the edge scene */
  {
    const double A[4] = {10.0, 7.5, 7.5, 10.0}, b[2] = {0.5, -1.0};
    orc_scene* q = orc_scene_quad(2, A, b, 0.3);
    const double th[2] = {0.3, -0.2};
    estimators(q, th, 2, 0.3, 16);
    solvers(q, th, 2, 0.3, 16);
    orc_scene_free(q);
    orc_scene* ng = orc_scene_neggauss(2, 1.0);
    estimators(ng, th, 2, 0.5, 16);
    solvers(ng, th, 2, 0.5, 16);
    orc_scene_free(ng);
    float tgt[64];
    for (int i = 0; i < 64; ++i) tgt[i] = 0.0f;
    orc_scene* e = orc_scene_edge(8, 8, 2, tgt);
    const double te[2] = {0.5, 0.4};
    estimators(e, te, 2, 0.1, 16);
    orc_scene_free(e);
    double ev[4], evec[4];
    CHECK(orc_jacobi_eig(2, A, ev, evec));
  }
  /* invalid arguments return errors and touch nothing */
  {
    orc_opts o = opts(ORC_AIS, 1, NULL);
    double g[2];
    if (orc_est_grad(NULL, NULL, 0.1, 4, 1, &o, g) == 0) ++fails;
  }
  if (!isfinite(acc)) ++fails;
  printf("%s\n", fails ? "sanitize driver: failures" : "sanitize driver ok");
  return fails ? 1 : 0;
}
