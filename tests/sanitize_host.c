/*
 * Drives the HIP library's host code where it runs without a device, for a
 * host-only build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers.py): option defaults, context creation on a host
 * with no usable GPU, and the argument checks of every entry point, which run
 * before any device work.  Each call must return its documented error, and the
 * run must finish without a sanitizer report or a leak.
 */
#include <stdio.h>
#include <string.h>

#include "hrest.h"

static int fails = 0;
#define EXPECT(call, want)                                                         \
  do {                                                                             \
    hr_status st_ = (call);                                                        \
    if (st_ != (want)) {                                                           \
      fprintf(stderr, "%s:%d: %s returned %d, expected %d\n", __FILE__, __LINE__, \
              #call, (int)st_, (int)(want));                                       \
      ++fails;                                                                     \
    }                                                                              \
  } while (0)

int main(void) {
  hr_opts o;
  hr_opts_default(&o);
  hr_ncg_opts no;
  hr_ncg_opts_default(&no);
  hr_optim_opts oo;
  hr_optim_opts_default(&oo);
  hr_batch_opts bo;
  hr_batch_opts_default(&bo);
  hr_server_opts so;
  hr_server_opts_default(&so);

  /* contexts: a negative device is an argument error; device 0 on a host
   * without a GPU is a device error (with one, the context is made and
   * released) */
  hr_ctx* ctx = NULL;
  EXPECT(hr_ctx_create(-1, &ctx), HR_EINVAL);
  EXPECT(hr_ctx_create(0, NULL), HR_EINVAL);
  hr_status st = hr_ctx_create(0, &ctx);
  if (st == HR_OK) {
    hr_ctx_destroy(ctx);
  } else if (st != HR_EDEVICE && st != HR_EINVAL) {
    fprintf(stderr, "hr_ctx_create(0) returned %d\n", (int)st);
    ++fails;
  }
  if (hr_last_error() == NULL) ++fails;
  hr_ctx_destroy(NULL);

  /* every entry point refuses missing handles and pointers */
  double theta[3] = {0.5, 0.5, 0.1}, v[3] = {1.0, 0.0, 0.0}, out[9];
  const double J[6] = {1, 0, 0, 1, 0, 0};
  void* p = NULL;
  hr_scene* sc = NULL;
  EXPECT(hr_ctx_set_stream(NULL, NULL), HR_EINVAL);
  EXPECT(hr_ctx_set_memory_budget(NULL, 1u << 20), HR_EINVAL);
  EXPECT(hr_ctx_synchronize(NULL), HR_EINVAL);
  EXPECT(hr_ctx_enable_timing(NULL, 1), HR_EINVAL);
  EXPECT(hr_ctx_reset_stats(NULL), HR_EINVAL);
  EXPECT(hr_dev_alloc(NULL, 16, &p), HR_EINVAL);
  EXPECT(hr_dev_free(NULL, p), HR_EINVAL);
  EXPECT(hr_memcpy(NULL, out, theta, 8, 0), HR_EINVAL);
  const float colors[3] = {1.0f, 0.5f, 0.25f}, target[12] = {0};
  EXPECT(hr_scene_disks(NULL, 2, 2, 3, 1, 3, NULL, colors, target, &sc), HR_EINVAL);
  EXPECT(hr_scene_quad(NULL, 1, theta, theta, 0.0, &sc), HR_EINVAL);
  EXPECT(hr_scene_neggauss(NULL, 2, 1.0, &sc), HR_EINVAL);
  hr_scene_destroy(NULL);
  if (hr_scene_nparams(NULL) > 0) ++fails;
  float img[12];
  EXPECT(hr_render(NULL, theta, 0, 0, 0, img), HR_EINVAL);
  EXPECT(hr_est_grad(NULL, theta, 0.1, 16, 1, &o, out), HR_EINVAL);
  EXPECT(hr_est_hessian(NULL, theta, 0.1, 16, 1, &o, out), HR_EINVAL);
  EXPECT(hr_est_hvp(NULL, theta, 0.1, 16, 1, v, &o, out), HR_EINVAL);
  EXPECT(hr_est_hvp_limit(NULL, theta, 0.1, 16, 1, v, &o, out), HR_EINVAL);
  EXPECT(hr_est_loss(NULL, theta, 0.1, 16, 1, &o, out), HR_EINVAL);
  EXPECT(hr_est_grad_greybox(NULL, theta, J, 2, 0.1, 16, 1, &o, out), HR_EINVAL);
  EXPECT(hr_est_hessian_greybox(NULL, theta, J, 2, 0.1, 16, 1, &o, out), HR_EINVAL);
  EXPECT(hr_est_hvp_greybox(NULL, theta, J, 2, 0.1, 16, 1, v, &o, out), HR_EINVAL);
  EXPECT(hr_est_grad_dev(NULL, theta, 0.1, 16, 1, &o, out), HR_EINVAL);
  EXPECT(hr_est_hessian_dev(NULL, theta, 0.1, 16, 1, &o, out), HR_EINVAL);
  EXPECT(hr_est_hvp_dev(NULL, theta, 0.1, 16, 1, v, &o, out), HR_EINVAL);
  EXPECT(hr_est_hvp_dev_noalloc(NULL, theta, 0.1, 16, 1, v, &o, out), HR_EINVAL);
  hr_ncg_report rep;
  EXPECT(hr_newton_cg_step(NULL, theta, 0.1, 16, 1, &no, &o, &rep), HR_EINVAL);
  EXPECT(hr_newton_cg_step_dev(NULL, theta, 0.1, 16, 1, &no, &o, &rep), HR_EINVAL);
  EXPECT(hr_optimize(NULL, theta, 16, 1, &oo, &o, out), HR_EINVAL);
  hr_batch* b = NULL;
  EXPECT(hr_batch_create(NULL, &bo, &b), HR_EINVAL);
  EXPECT(hr_batch_run(NULL, NULL, 0), HR_EINVAL);
  hr_batch_report br;
  EXPECT(hr_batch_report_get(NULL, &br), HR_EINVAL);
  hr_batch_destroy(NULL);
  hr_server* srv = NULL;
  EXPECT(hr_server_create(NULL, &so, &srv), HR_EINVAL);
  uint64_t ticket = 0;
  hr_query q;
  memset(&q, 0, sizeof q);
  EXPECT(hr_submit(NULL, &q, &ticket), HR_EINVAL);
  EXPECT(hr_wait(NULL, 1, out, NULL), HR_EINVAL);
  EXPECT(hr_wait_any(NULL, 1.0, &ticket), HR_EINVAL);
  hr_server_stats ss;
  EXPECT(hr_server_stats_get(NULL, &ss), HR_EINVAL);
  hr_server_destroy(NULL);

  printf("%s\n", fails ? "sanitize host driver: failures" : "sanitize host driver ok");
  return fails ? 1 : 0;
}
