/*
 * orc.c -- CPU FP64 oracle (test infrastructure only; see orc.h).
 *
 * Paper: Z. Wang, M. Fischer, T. Ritschel, "Stochastic Gradient Estimation for
 * Higher-order Differentiable Rendering", ICCV 2025 (arXiv 2412.03489).
 *
 * This file restates the paper's estimators in the plainest form that is still
 * usable: one sample at a time, every element of every kernel written out, no
 * blocking, no fusion, no reordering of sums beyond sample order.  Where the
 * paper is silent or garbled, the reading taken is stated next to the code.
 *
 * Parity pins (what checks this file against something other than itself) live
 * in tests/test_oracle_*.py: Philox4x32-10 known-answer vectors and an
 * independent implementation, quadrature of lobe masses, CDF anchors, KS
 * tests, closed forms for quadratic, negated-Gaussian, half-plane and corner
 * scenes, exact smoothed derivatives of the one-disk scene by contour
 * quadrature, hand-built disk images (painter's order, colours, radius from
 * theta, r <= 0, strict edges), the exact smoothed loss of overlapping RGB
 * disks with radius parameters, and the path tracer's ray hits, shadows,
 * direct light (Lambert's polygon formula) and one-bounce indirect light
 * (quadrature over the sphere's surface).
 */
#include "orc.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

/* ========================================================================= */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random numbers:
 * as easy as 1, 2, 3").  Round: two 32x32->64 multiplications of counter words
 * 0 and 2 by the round multipliers; the high halves are XORed with the other
 * counter words and the key; the key is bumped by the Weyl constants between
 * rounds.  Ten rounds.                                                       */
/* ========================================================================= */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += W0; k1 += W1; }
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_words(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                         uint32_t out[4]) {
  uint32_t ctr[4] = {a, b, c, d};
  uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* open-interval uniform from one 32-bit word: (w + 1/2) / 2^32, exact in FP64 */
static double unif(uint32_t w) { return ldexp((double)w + 0.5, -32); }

/* Counter tags (the paper fixes no random-number layout). */
#define TAG_AIS   0x7FFFFFFFu
#define TAG_GAUSS 0x7FFFFFFEu
#define TAG_PIX   0x80000000u
#define DIM_SELECT 0xFFFFFFFFu

/* ========================================================================= */
/* One-dimensional samplers                                                  */
/* ========================================================================= */

/* Section "Gradients", Sampling: inverse CDF of the positivised, normalised
 * derivative-of-Gaussian lobe pair.  The printed formula has the argument of the
 * logarithm and the sign garbled; the CDF of |u| e^{-u^2/2s^2}/(2 s^2) is
 * (1/2) e^{-u^2/2s^2} for u<0 and 1 - (1/2) e^{-u^2/2s^2} for u>0, whose inverse
 * is used here.  The branch is decided on the integer word (xi <= 1/2). */
double orc_grad_lobe_icdf(uint32_t w, double sigma) {
  if (w < 0x80000000u) {
    double two_xi = ldexp((double)w + 0.5, -31);               /* 2 xi       */
    return -sigma * sqrt(-2.0 * log(two_xi));
  } else {
    double two_1mxi = ldexp((double)(0xFFFFFFFFu - w) + 0.5, -31);  /* 2(1-xi) */
    return sigma * sqrt(-2.0 * log(two_1mxi));
  }
}

/* Lambert W by Halley's iteration (Corless, Gonnet, Hare, Jeffrey, Knuth 1996,
 * "On the Lambert W function"), branch 0 or -1, for z in [-1/e, 0).
 * Start: branch-point series in p = sqrt(2(e z + 1)) near -1/e; log asymptotics
 * of W_{-1} near 0^-; z itself for W_0 near 0. */
double orc_lambertw(double z, int branch) {
  /* e z + 1, which vanishes at the branch point, from e split into a double
   * and its rounding remainder so that the distance to -1/e keeps its digits */
  const double E = 2.71828182845904523536, E_LO = 1.4456468917292502e-16;
  double t = fma(E, z, 1.0) + E_LO * z;
  if (t <= 0.0) return -1.0;
  double p = sqrt(2.0 * t);
  double w;
  if (branch == 0) {
    if (t < 0.25) w = -1.0 + p - p * p / 3.0 + 11.0 / 72.0 * p * p * p;
    else w = z;  /* |W_0(z)| small here; Halley converges from z */
  } else {
    if (t < 0.25) w = -1.0 - p - p * p / 3.0 - 11.0 / 72.0 * p * p * p;
    else {
      double L1 = log(-z), L2 = log(-L1);
      w = L1 - L2 + L2 / L1;
    }
  }
  for (int it = 0; it < 64; ++it) {
    double ew = exp(w);
    double f = w * ew - z;
    double wp1 = w + 1.0;
    if (wp1 == 0.0) break;
    double denom = ew * wp1 - (w + 2.0) * f / (2.0 * wp1);
    if (denom == 0.0) break;
    double dw = f / denom;
    w -= dw;
    if (fabs(dw) <= 1e-16 * (1.0 + fabs(w))) break;
  }
  return w;
}

/* Section "Hessians", Sampling: three-branch CDF of the positivised second
 * derivative of the 1-D Gaussian, scaled to 1/4 at -sigma. */
double orc_hdiag_cdf(double u, double sigma) {
  double e = exp(0.5 - u * u / (2.0 * sigma * sigma));
  if (u < -sigma) return -(u / (4.0 * sigma)) * e;
  if (u <= sigma) return 0.5 + (u / (4.0 * sigma)) * e;
  return 1.0 - (u / (4.0 * sigma)) * e;
}

/* Inverse of orc_hdiag_cdf.  The paper tabulates it numerically; with
 * s = u^2/sigma^2 each branch reads s e^{-s} = 16 y^2 / e (y = xi, xi - 1/2 or
 * 1 - xi), so s = -W(-16 y^2/e): W_{-1} on the tails (s > 1), W_0 inside. */
double orc_hdiag_icdf(uint32_t w, double sigma) {
  const double E = 2.71828182845904523536;
  double xi = unif(w);
  double s;
  if (w < 0x40000000u) {                      /* xi < 1/4: left tail         */
    s = -orc_lambertw(-16.0 * xi * xi / E, -1);
    return -sigma * sqrt(s);
  } else if (w >= 0xC0000000u) {              /* xi > 3/4: right tail        */
    double om = ldexp((double)(0xFFFFFFFFu - w) + 0.5, -32);   /* 1 - xi exact */
    s = -orc_lambertw(-16.0 * om * om / E, -1);
    return sigma * sqrt(s);
  } else {                                    /* inner lobe                  */
    double d = xi - 0.5;
    s = -orc_lambertw(-16.0 * d * d / E, 0);
    if (s < 0.0) s = 0.0;
    return (d < 0.0 ? -sigma : sigma) * sqrt(s);
  }
}

/* ========================================================================= */
/* Scenes                                                                    */
/* ========================================================================= */
enum { SC_DISKS = 0, SC_PT = 1, SC_QUAD = 2, SC_NEGGAUSS = 3, SC_EDGE = 4 };

struct orc_scene {
  int kind;
  int n;             /* number of parameters */
  /* image scenes */
  int W, H, C;
  float* target;     /* H*W*C, row-major (y, x, channel) */
  /* disks */
  int D, ppd;
  float* radius;     /* D (ppd == 2) */
  float* colors;     /* D*C */
  /* path tracer */
  int spp, nspheres;
  double* desc;
  /* analytic */
  double *A, *b, c, s1;
};

static float* copy_f(const float* p, size_t n) {
  if (!p || n == 0) return NULL;
  float* q = (float*)malloc(n * sizeof(float));
  memcpy(q, p, n * sizeof(float));
  return q;
}
static double* copy_d(const double* p, size_t n) {
  if (!p || n == 0) return NULL;
  double* q = (double*)malloc(n * sizeof(double));
  memcpy(q, p, n * sizeof(double));
  return q;
}

orc_scene* orc_scene_disks(int W, int H, int C, int D, int ppd, const float* radius,
                           const float* colors, const float* target) {
  if (W <= 0 || H <= 0 || C <= 0 || D <= 0 || (ppd != 2 && ppd != 3)) return NULL;
  if (ppd == 2 && !radius) return NULL;
  orc_scene* sc = (orc_scene*)calloc(1, sizeof(orc_scene));
  sc->kind = SC_DISKS; sc->W = W; sc->H = H; sc->C = C; sc->D = D; sc->ppd = ppd;
  sc->n = D * ppd;
  sc->radius = ppd == 2 ? copy_f(radius, (size_t)D) : NULL;
  sc->colors = copy_f(colors, (size_t)D * C);
  sc->target = copy_f(target, (size_t)W * H * C);
  return sc;
}

/* desc: eye[3], look_at[3], vfov_deg, light_side, Le, ground_albedo[3], then per
 * sphere: center[3], radius, albedo[3].  Parameters: light centre xyz, then
 * the centre xyz of sphere 0 (its stored centre is ignored). */
orc_scene* orc_scene_pt(int W, int H, int spp, int nspheres, const double* desc,
                        const float* target) {
  if (W <= 0 || H <= 0 || spp <= 0 || nspheres <= 0 || !desc) return NULL;
  orc_scene* sc = (orc_scene*)calloc(1, sizeof(orc_scene));
  sc->kind = SC_PT; sc->W = W; sc->H = H; sc->C = 3; sc->spp = spp;
  sc->nspheres = nspheres; sc->n = 6;
  sc->desc = copy_d(desc, (size_t)(12 + 7 * nspheres));
  sc->target = copy_f(target, (size_t)W * H * 3);
  return sc;
}

orc_scene* orc_scene_quad(int n, const double* A, const double* b, double c) {
  if (n <= 0 || !A) return NULL;
  orc_scene* sc = (orc_scene*)calloc(1, sizeof(orc_scene));
  sc->kind = SC_QUAD; sc->n = n;
  sc->A = copy_d(A, (size_t)n * n);
  sc->b = (double*)calloc((size_t)n, sizeof(double));
  if (b) memcpy(sc->b, b, (size_t)n * sizeof(double));
  sc->c = c;
  return sc;
}

orc_scene* orc_scene_neggauss(int n, double s1) {
  if (n <= 0 || !(s1 > 0)) return NULL;
  orc_scene* sc = (orc_scene*)calloc(1, sizeof(orc_scene));
  sc->kind = SC_NEGGAUSS; sc->n = n; sc->s1 = s1;
  return sc;
}

orc_scene* orc_scene_edge(int W, int H, int n, const float* target) {
  if (W <= 0 || H <= 0 || (n != 1 && n != 2)) return NULL;
  orc_scene* sc = (orc_scene*)calloc(1, sizeof(orc_scene));
  sc->kind = SC_EDGE; sc->W = W; sc->H = H; sc->C = 1; sc->n = n;
  sc->target = copy_f(target, (size_t)W * H);
  return sc;
}

void orc_scene_free(orc_scene* sc) {
  if (!sc) return;
  free(sc->target); free(sc->radius); free(sc->colors); free(sc->desc);
  free(sc->A); free(sc->b);
  free(sc);
}

int orc_scene_nparams(const orc_scene* sc) { return sc ? sc->n : -1; }

/* ---- disk rasterizer: pixel centre ((x+1/2)/W, (y+1/2)/H), y down; a disk
 * covers a centre iff its radius is positive and the squared distance is below
 * r^2; painter's order by index (later disks on top); background 0. ---- */
static void render_disks(const orc_scene* sc, const double* th, double* out) {
  for (int y = 0; y < sc->H; ++y) {
    for (int x = 0; x < sc->W; ++x) {
      double px = (x + 0.5) / sc->W, py = (y + 0.5) / sc->H;
      int top = -1;
      for (int k = 0; k < sc->D; ++k) {
        double cx = th[k * sc->ppd + 0];
        double cy = th[k * sc->ppd + 1];
        double r = sc->ppd == 3 ? th[k * sc->ppd + 2] : (double)sc->radius[k];
        double dx = px - cx, dy = py - cy;
        if (r > 0.0 && dx * dx + dy * dy < r * r) top = k;
      }
      for (int ch = 0; ch < sc->C; ++ch)
        out[((size_t)y * sc->W + x) * sc->C + ch] =
            top >= 0 ? (double)sc->colors[top * sc->C + ch] : 0.0;
    }
  }
}

/* ---- edge scene: I = 1 where px < theta_0 (and py < theta_1 for n = 2) ---- */
static void render_edge(const orc_scene* sc, const double* th, double* out) {
  for (int y = 0; y < sc->H; ++y)
    for (int x = 0; x < sc->W; ++x) {
      double px = (x + 0.5) / sc->W, py = (y + 0.5) / sc->H;
      int in = px < th[0];
      if (sc->n == 2) in = in && (py < th[1]);
      out[(size_t)y * sc->W + x] = in ? 1.0 : 0.0;
    }
}

/* ---- path tracer (section "Background": Monte Carlo light transport with
 * standard light and BRDF sampling).  Diffuse spheres on the plane y = 0, one
 * one-sided square light facing -y.  Per path: camera ray; emission only if the
 * camera ray sees the light; next-event estimation towards a uniform point on
 * the light at the first and second surface hits; one cosine-weighted bounce;
 * no Russian roulette; black background. ---- */
typedef struct { double x, y, z; } v3;
static v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 cross(v3 a, v3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static v3 normalize(v3 a) { return scl(a, 1.0 / sqrt(dot(a, a))); }

#define PT_EPS 1e-4
#define PT_TMIN 1e-6

typedef struct {
  const orc_scene* sc;
  v3 light;       /* light centre */
  v3 s0;          /* sphere-0 centre */
} pt_ctx;

static v3 sphere_center(const pt_ctx* c, int i) {
  if (i == 0) return c->s0;
  const double* s = c->sc->desc + 12 + 7 * i;
  return mk(s[0], s[1], s[2]);
}
static double sphere_radius(const pt_ctx* c, int i) { return c->sc->desc[12 + 7 * i + 3]; }

/* closest hit: returns object id (-1 none, 0..ns-1 sphere, ns plane, ns+1 light) */
static int pt_intersect(const pt_ctx* c, v3 o, v3 d, double* tbest) {
  int ns = c->sc->nspheres, id = -1;
  double best = 1e300;
  for (int i = 0; i < ns; ++i) {
    v3 oc = sub(o, sphere_center(c, i));
    double r = sphere_radius(c, i);
    double b = dot(oc, d), cc = dot(oc, oc) - r * r, disc = b * b - cc;
    if (disc < 0.0) continue;
    double sq = sqrt(disc);
    double t = -b - sq;
    if (!(t > PT_TMIN)) t = -b + sq;
    if (t > PT_TMIN && t < best) { best = t; id = i; }
  }
  if (d.y != 0.0) {
    double t = -o.y / d.y;
    if (t > PT_TMIN && t < best) { best = t; id = ns; }
    double half = 0.5 * c->sc->desc[7];
    double tl = (c->light.y - o.y) / d.y;
    if (tl > PT_TMIN && tl < best) {
      v3 p = add(o, scl(d, tl));
      if (fabs(p.x - c->light.x) <= half && fabs(p.z - c->light.z) <= half) {
        best = tl; id = ns + 1;
      }
    }
  }
  *tbest = best;
  return id;
}

static int pt_occluded(const pt_ctx* c, v3 o, v3 d, double dist) {
  int ns = c->sc->nspheres;
  double tmax = dist - PT_EPS;
  for (int i = 0; i < ns; ++i) {
    v3 oc = sub(o, sphere_center(c, i));
    double r = sphere_radius(c, i);
    double b = dot(oc, d), cc = dot(oc, oc) - r * r, disc = b * b - cc;
    if (disc < 0.0) continue;
    double sq = sqrt(disc);
    double t = -b - sq;
    if (!(t > PT_TMIN)) t = -b + sq;
    if (t > PT_TMIN && t < tmax) return 1;
  }
  if (d.y != 0.0) {
    double t = -o.y / d.y;
    if (t > PT_TMIN && t < tmax) return 1;
  }
  return 0;
}

/* direct light from the square source at surface origin o (already offset)
 * with normal n, for the light point chosen by uniforms (u1, u2); returns the
 * scalar factor Le cos_x cos_l A / d^2 / pi (times albedo by the caller). */
static double pt_nee(const pt_ctx* c, v3 o, v3 n, double u1, double u2) {
  double side = c->sc->desc[7], Le = c->sc->desc[8];
  v3 y = mk(c->light.x + (u1 - 0.5) * side, c->light.y, c->light.z + (u2 - 0.5) * side);
  v3 wv = sub(y, o);
  double d2 = dot(wv, wv);
  double dist = sqrt(d2);
  v3 wi = scl(wv, 1.0 / dist);
  double cosx = dot(n, wi);
  double cosl = wi.y;   /* light normal (0,-1,0): cos at the light = -n_l . wi */
  if (!(cosx > 0.0) || !(cosl > 0.0)) return 0.0;
  if (pt_occluded(c, o, wi, dist)) return 0.0;
  return Le * cosx * cosl * side * side / d2 / PI;
}

static void pt_surface(const pt_ctx* c, int id, v3 x, v3* n, double alb[3]) {
  int ns = c->sc->nspheres;
  if (id < ns) {
    *n = scl(sub(x, sphere_center(c, id)), 1.0 / sphere_radius(c, id));
    const double* s = c->sc->desc + 12 + 7 * id;
    alb[0] = s[4]; alb[1] = s[5]; alb[2] = s[6];
  } else {
    *n = mk(0.0, 1.0, 0.0);
    alb[0] = c->sc->desc[9]; alb[1] = c->sc->desc[10]; alb[2] = c->sc->desc[11];
  }
}

/* orthonormal basis around a unit normal (Duff et al., JCGT 2017) */
static void onb(v3 n, v3* b1, v3* b2) {
  double sign = copysign(1.0, n.z);
  double a = -1.0 / (sign + n.z);
  double b = n.x * n.y * a;
  *b1 = mk(1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x);
  *b2 = mk(b, sign + n.y * n.y * a, -n.y);
}

static void pt_radiance(const pt_ctx* c, v3 eye, v3 d, const double u[8], double L[3]) {
  L[0] = L[1] = L[2] = 0.0;
  double t;
  int id = pt_intersect(c, eye, d, &t);
  int ns = c->sc->nspheres;
  if (id < 0) return;
  if (id == ns + 1) {
    if (d.y > 0.0) L[0] = L[1] = L[2] = c->sc->desc[8];
    return;
  }
  v3 x = add(eye, scl(d, t)), n;
  double alb[3];
  pt_surface(c, id, x, &n, alb);
  v3 o1 = add(x, scl(n, PT_EPS));
  double e1 = pt_nee(c, o1, n, u[2], u[3]);
  for (int k = 0; k < 3; ++k) L[k] += alb[k] * e1;
  /* cosine-weighted bounce (Malley): r = sqrt(u), phi = 2 pi u', z = sqrt(1-u) */
  double r = sqrt(u[4]), phi = 2.0 * PI * u[5];
  v3 b1, b2;
  onb(n, &b1, &b2);
  v3 dir = add(add(scl(b1, r * cos(phi)), scl(b2, r * sin(phi))), scl(n, sqrt(1.0 - u[4])));
  double t2;
  int id2 = pt_intersect(c, o1, dir, &t2);
  if (id2 < 0 || id2 == ns + 1) return;   /* bounce sees sky or light: path ends */
  v3 x2 = add(o1, scl(dir, t2)), n2;
  double alb2[3];
  pt_surface(c, id2, x2, &n2, alb2);
  v3 o2 = add(x2, scl(n2, PT_EPS));
  double e2 = pt_nee(c, o2, n2, u[6], u[7]);
  for (int k = 0; k < 3; ++k) L[k] += alb[k] * alb2[k] * e2;
}

static void render_pt(const orc_scene* sc, const double* th, uint64_t seed, uint32_t s,
                      int spp, double* out) {
  pt_ctx c;
  c.sc = sc;
  c.light = mk(th[0], th[1], th[2]);
  c.s0 = mk(th[3], th[4], th[5]);
  const double* dsc = sc->desc;
  v3 eye = mk(dsc[0], dsc[1], dsc[2]), look = mk(dsc[3], dsc[4], dsc[5]);
  v3 fwd = normalize(sub(look, eye));
  v3 right = normalize(cross(fwd, mk(0.0, 1.0, 0.0)));
  v3 upv = cross(right, fwd);
  double th_half = tan(0.5 * dsc[6] * PI / 180.0);
  double aspect = (double)sc->W / (double)sc->H;
  for (int y = 0; y < sc->H; ++y) {
    for (int x = 0; x < sc->W; ++x) {
      uint32_t pix = (uint32_t)(y * sc->W + x);
      double acc[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < spp; ++k) {
        uint32_t wa[4], wb[4];
        philox_words(seed, s, pix, (uint32_t)(16 * k + 0), TAG_PIX, wa);
        philox_words(seed, s, pix, (uint32_t)(16 * k + 1), TAG_PIX, wb);
        double u[8] = {unif(wa[0]), unif(wa[1]), unif(wa[2]), unif(wa[3]),
                       unif(wb[0]), unif(wb[1]), unif(wb[2]), unif(wb[3])};
        double sx = (2.0 * (x + u[0]) / sc->W - 1.0) * th_half * aspect;
        double sy = (1.0 - 2.0 * (y + u[1]) / sc->H) * th_half;
        v3 d = normalize(add(add(fwd, scl(right, sx)), scl(upv, sy)));
        double L[3];
        pt_radiance(&c, eye, d, u, L);
        for (int ch = 0; ch < 3; ++ch) acc[ch] += L[ch];
      }
      for (int ch = 0; ch < 3; ++ch) out[(size_t)pix * 3 + ch] = acc[ch] / spp;
    }
  }
}

/* Hooks of the path tracer for the tests' pins: the closest hit along a ray
 * (object id as pt_intersect: -1 none, 0..ns-1 sphere, ns plane, ns+1 light;
 * *t its distance), and the radiance of one path from o along the unit
 * direction d with the eight uniforms u (2-3: light point at the first hit,
 * 4-5: bounce, 6-7: light point at the second hit; 0-1 are the pixel jitter
 * and unused here). */
static pt_ctx pt_ctx_of(const orc_scene* sc, const double* th) {
  pt_ctx c;
  c.sc = sc;
  c.light = mk(th[0], th[1], th[2]);
  c.s0 = mk(th[3], th[4], th[5]);
  return c;
}

int orc_pt_trace(const orc_scene* sc, const double* theta, const double* o, const double* d,
                 double* t) {
  if (!sc || sc->kind != SC_PT || !theta || !o || !d || !t) return -2;
  pt_ctx c = pt_ctx_of(sc, theta);
  return pt_intersect(&c, mk(o[0], o[1], o[2]), mk(d[0], d[1], d[2]), t);
}

int orc_pt_path(const orc_scene* sc, const double* theta, const double* o, const double* d,
                const double* u, double* L) {
  if (!sc || sc->kind != SC_PT || !theta || !o || !d || !u || !L) return -1;
  pt_ctx c = pt_ctx_of(sc, theta);
  pt_radiance(&c, mk(o[0], o[1], o[2]), mk(d[0], d[1], d[2]), u, L);
  return 0;
}

int orc_render(const orc_scene* sc, const double* theta, uint64_t seed, uint32_t s,
               int spp_override, double* out) {
  if (!sc || !theta || !out) return -1;
  switch (sc->kind) {
    case SC_DISKS: render_disks(sc, theta, out); return 0;
    case SC_EDGE: render_edge(sc, theta, out); return 0;
    case SC_PT:
      render_pt(sc, theta, seed, s, spp_override > 0 ? spp_override : sc->spp, out);
      return 0;
    default: return -4;
  }
}

/* Loss: mean squared error over all H*W*C values against the stored target
 * (the paper's image loss; its normalisation is not stated, the mean is used).
 * Analytic scenes return their function value. */
double orc_loss(const orc_scene* sc, const double* theta, uint64_t seed, uint32_t s) {
  if (sc->kind == SC_QUAD) {
    double f = sc->c;
    for (int i = 0; i < sc->n; ++i) {
      f += sc->b[i] * theta[i];
      for (int j = 0; j < sc->n; ++j) f += 0.5 * theta[i] * sc->A[i * sc->n + j] * theta[j];
    }
    return f;
  }
  if (sc->kind == SC_NEGGAUSS) {
    double r2 = 0.0;
    for (int i = 0; i < sc->n; ++i) r2 += theta[i] * theta[i];
    return -pow(2.0 * PI * sc->s1 * sc->s1, -0.5 * sc->n) * exp(-r2 / (2.0 * sc->s1 * sc->s1));
  }
  size_t P = (size_t)sc->W * sc->H * sc->C;
  double* img = (double*)malloc(P * sizeof(double));
  orc_render(sc, theta, seed, s, 0, img);
  double acc = 0.0;
  for (size_t i = 0; i < P; ++i) {
    double e = img[i] - (double)sc->target[i];
    acc += e * e;
  }
  free(img);
  return acc / (double)P;
}

/* ========================================================================= */
/* Kernels of the smoothed differential operators                            */
/* ========================================================================= */
/* Element sets: gradient K = n (element m = dimension m); Hessian K = n(n+1)/2
 * over i <= j (section "Hessians": the symmetry is exploited), enumerated row
 * by row: (0,0), (0,1), ..., (0,n-1), (1,1), ...  The (i, j) of every element
 * is listed once per estimator call in a table. */
typedef struct { int* i; int* j; int K; } tri_table;

static tri_table tri_make(int n) {
  tri_table t;
  t.K = n * (n + 1) / 2;
  t.i = (int*)malloc((size_t)t.K * sizeof(int));
  t.j = (int*)malloc((size_t)t.K * sizeof(int));
  int idx = 0;
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) { t.i[idx] = i; t.j[idx] = j; ++idx; }
  return t;
}
static void tri_free(tri_table* t) { free(t->i); free(t->j); }

static void hess_ij(int n, int m, int* pi, int* pj) {
  int idx = 0;
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      if (idx == m) { *pi = i; *pj = j; return; }
      ++idx;
    }
  *pi = *pj = -1;
}

/* L1 masses of the 1-D kernel factors times the Gaussian:
 *   gradient  |d/du N(u)|      -> sqrt(2/pi)/sigma
 *   diagonal  |d2/du2 N(u)|    -> 4 e^{-1/2} / (sigma^2 sqrt(2 pi))
 *   off-diag  product of two gradient factors -> (sqrt(2/pi)/sigma)^2 */
static double Z_grad(double sg) { return sqrt(2.0 / PI) / sg; }
static double Z_diag(double sg) { return 4.0 * exp(-0.5) / (sg * sg * sqrt(2.0 * PI)); }

/* kernel factor d_m(tau) such that D kappa_m(tau) = d_m(tau) N(tau):
 * gradient eq. (gradient kernel): -tau_m / sigma^2;
 * Hessian (Hessian kernel): tau_i^2/sigma^4 - 1/sigma^2 on the diagonal and
 * tau_i tau_j / sigma^4 off it. */
static double kfac(int hess, const tri_table* T, int m, const double* tau, double sg) {
  double s2 = sg * sg;
  if (!hess) return -tau[m] / s2;
  int i = T->i[m], j = T->j[m];
  if (i == j) return tau[i] * tau[i] / (s2 * s2) - 1.0 / s2;
  return tau[i] * tau[j] / (s2 * s2);
}
static double kmass(int hess, const tri_table* T, int m, double sg) {
  if (!hess) return Z_grad(sg);
  return T->i[m] == T->j[m] ? Z_diag(sg) : Z_grad(sg) * Z_grad(sg);
}

/* ========================================================================= */
/* Drawing tau for one sample                                                */
/* ========================================================================= */
/* Per sample s and dimension j one Philox block (s, j, 0, tag): words 0 and 1
 * give a Box-Muller Gaussian (Box & Muller 1958), word 2 the lobe uniform.
 * The sampled element's own dimensions are drawn from its lobe distribution,
 * every other dimension from the Gaussian (section "Gradients", Sampling, and
 * the marginalisation appendix).  The aggregate sampler first draws the element
 * uniformly from the selector block (s, 0xFFFFFFFF, 0, tag). */
/* per-element streams: IS, and the FR22 comparator (appendix on the gradient
 * derivation: FR22 blurs only the dimension it differentiates, so every other
 * dimension of its draw is zero) */
static int per_element(int sampler) { return sampler == ORC_IS || sampler == ORC_FR22; }

/* Aggregate Hessian mixtures (section "Aggregate"): the element is either one
 * of the K unique (i <= j) elements, or one of the n^2 ordered pairs (i, j),
 * whose kernel and density are those of the unique element (min, max).  Under
 * the n^2 mixture an off-diagonal element is chosen twice as often as a
 * diagonal one. */
static int tri_index(int n, int i, int j) {
  int a = i < j ? i : j, b = i < j ? j : i;
  return a * n - a * (a - 1) / 2 + (b - a);
}

static void draw(int hess, int n, double sg, uint64_t seed, uint32_t s, int sampler,
                 int mix_n2, int stream, double* tau, int* elem) {
  int K = hess ? n * (n + 1) / 2 : n;
  uint32_t tag = per_element(sampler) ? (uint32_t)stream
                                      : (sampler == ORC_AIS ? TAG_AIS : TAG_GAUSS);
  uint32_t* lobe = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
  for (int j = 0; j < n; ++j) {
    uint32_t w[4];
    philox_words(seed, s, (uint32_t)j, 0u, tag, w);
    tau[j] = sg * sqrt(-2.0 * log(unif(w[0]))) * cos(2.0 * PI * unif(w[1]));
    lobe[j] = w[2];
  }
  int m = -1;
  if (per_element(sampler)) m = stream;
  if (sampler == ORC_FR22)
    for (int j = 0; j < n; ++j) tau[j] = 0.0;
  if (sampler == ORC_AIS) {
    uint32_t w[4];
    philox_words(seed, s, DIM_SELECT, 0u, tag, w);
    if (hess && mix_n2) {
      int pair = (int)(((uint64_t)w[0] * (uint64_t)n * (uint64_t)n) >> 32);
      m = tri_index(n, pair / n, pair % n);
    } else {
      m = (int)(((uint64_t)w[0] * (uint64_t)K) >> 32);
    }
  }
  if (m >= 0) {
    if (!hess) {
      tau[m] = orc_grad_lobe_icdf(lobe[m], sg);
    } else {
      int i, j;
      hess_ij(n, m, &i, &j);
      if (i == j) tau[i] = orc_hdiag_icdf(lobe[i], sg);
      else {
        tau[i] = orc_grad_lobe_icdf(lobe[i], sg);
        tau[j] = orc_grad_lobe_icdf(lobe[j], sg);
      }
    }
  }
  free(lobe);
  *elem = m;
}

int orc_draw_tau(int what, int n, double sigma, uint64_t seed, uint32_t s, int sampler,
                 int mix_n2, int stream, double* tau, int* element) {
  if (n <= 0 || !(sigma > 0) || !tau || (mix_n2 != 0 && mix_n2 != 1)) return -1;
  int e;
  draw(what == 1, n, sigma, seed, s, sampler, mix_n2, stream, tau, &e);
  if (element) *element = e;
  return 0;
}

/* Aggregate mixture density over the Gaussian: q = (1/K) sum_k |d_k| / Z_k
 * over the K elements, or for the n^2 Hessian mixture (1/n^2) times the sum
 * over all ordered pairs (i, j) of |d_ij| / Z_ij. */
static double mixture_q(int hess, int mix_n2, int n, const tri_table* T, int K,
                        const double* tau, double sg) {
  double q = 0.0;
  if (hess && mix_n2) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        int m = tri_index(n, i, j);
        q += fabs(kfac(1, T, m, tau, sg)) / kmass(1, T, m, sg);
      }
    return q / ((double)n * (double)n);
  }
  for (int k = 0; k < K; ++k) q += fabs(kfac(hess, T, k, tau, sg)) / kmass(hess, T, k, sg);
  return q / K;
}

/* Weights of all K elements for the draw tau:
 *  IS   : d_m N / p_m = sgn(d_m) Z_m
 *  AIS  : d_m N / q   with q the mixture density above (the "average of all
 *         stencils")
 *  GAUSS: d_m N / N = d_m */
static void weights(int hess, int mix_n2, int n, const tri_table* T, int K, const double* tau,
                    double sg, int sampler, double* w) {
  double q = 1.0;
  if (sampler == ORC_AIS) q = mixture_q(hess, mix_n2, n, T, K, tau, sg);
  for (int m = 0; m < K; ++m) {
    double dm = kfac(hess, T, m, tau, sg);
    if (sampler == ORC_GAUSS) w[m] = dm;
    else if (per_element(sampler))
      w[m] = (dm > 0.0 ? 1.0 : (dm < 0.0 ? -1.0 : 0.0)) * kmass(hess, T, m, sg);
    else w[m] = dm / q;
  }
}

/* ========================================================================= */
/* Estimator loop                                                            */
/* ========================================================================= */
enum { W_GRAD = 0, W_HESS = 1, W_HVP = 2, W_HVPL = 3 };

typedef struct {
  const orc_scene* sc;
  int what, n, K, sampler, mix_n2, A, nsh;
  const double* theta;
  double sg, h;
  const double* u;       /* HVP unit direction */
  const double* v;       /* HVP-limit direction */
  double vnorm;
  uint64_t N, seed, s0;
  double* contrib;       /* per item: K values (AIS/GAUSS) or 1 value (IS) */
  double* dbg;
  const tri_table* T;    /* (i, j) of the Hessian elements */
  uint64_t lo, hi;       /* item range for one worker */
} job_t;

static void run_item(const job_t* J, uint64_t item) {
  int n = J->n;
  uint64_t stream = per_element(J->sampler) ? item / J->N : 0;
  uint64_t sl = per_element(J->sampler) ? item % J->N : item;
  uint32_t s = (uint32_t)(J->s0 + sl);
  int hess_kernel = (J->what == W_HESS || J->what == W_HVPL);
  double* tau = (double*)malloc((size_t)n * sizeof(double));
  double* ntau = (double*)malloc((size_t)n * sizeof(double));
  double* p = (double*)malloc((size_t)n * sizeof(double));
  int elem;
  draw(hess_kernel, n, J->sg, J->seed, s, J->sampler, J->mix_n2, (int)stream, tau, &elem);
  for (int j = 0; j < n; ++j) ntau[j] = -tau[j];

  /* losses: f(theta - a tau) [+- h u for the HVP], a = +1 then -1 */
  double f[2][2];
  for (int ai = 0; ai < J->A; ++ai) {
    double a = ai == 0 ? 1.0 : -1.0;
    for (int hi = 0; hi < J->nsh; ++hi) {
      for (int j = 0; j < n; ++j) {
        double base = J->theta[j];
        if (J->what == W_HVP) base = base + (hi == 0 ? 1.0 : -1.0) * J->h * J->u[j];
        p[j] = base - a * tau[j];
      }
      f[ai][hi] = orc_loss(J->sc, p, J->seed, s);
      if (J->dbg) {
        uint64_t r = ((stream * J->N + sl) * (uint64_t)J->A + ai) * (uint64_t)J->nsh + hi;
        J->dbg[r] = f[ai][hi];
      }
    }
  }

  if (J->what == W_HVPL) {
    /* weight of output i: sum_j v_j d_ij(tau) / q(tau), with the symmetric
     * Hessian kernel (d_ji = d_ij) and the aggregate mixture over i <= j */
    double q = 1.0;
    if (J->sampler == ORC_AIS) q = mixture_q(1, J->mix_n2, n, J->T, J->K, tau, J->sg);
    double fs = 0.0;
    for (int ai = 0; ai < J->A; ++ai) fs += f[ai][0];
    double* c = J->contrib + item * (uint64_t)n;
    for (int i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += J->v[j] * kfac(1, J->T, tri_index(n, i, j), tau, J->sg);
      /* the Hessian kernel is even in tau, so both antithetic renders share it */
      c[i] = acc / q * fs;
    }
  } else {
    double* w[2];
    w[0] = (double*)malloc((size_t)J->K * sizeof(double));
    w[1] = (double*)malloc((size_t)J->K * sizeof(double));
    for (int ai = 0; ai < J->A; ++ai)
      weights(hess_kernel, J->mix_n2, n, J->T, J->K, ai == 0 ? tau : ntau, J->sg, J->sampler,
              w[ai]);
    double fv[2];
    for (int ai = 0; ai < J->A; ++ai)
      fv[ai] = J->what == W_HVP ? J->vnorm * (f[ai][0] - f[ai][1]) / (2.0 * J->h) : f[ai][0];
    if (per_element(J->sampler)) {
      int m = (int)stream;
      double val = 0.0;
      for (int ai = 0; ai < J->A; ++ai) val += w[ai][m] * fv[ai];
      J->contrib[item] = val;
    } else {
      double* c = J->contrib + item * (uint64_t)J->K;
      for (int m = 0; m < J->K; ++m) {
        double val = 0.0;
        for (int ai = 0; ai < J->A; ++ai) val += w[ai][m] * fv[ai];
        c[m] = val;
      }
    }
    free(w[0]); free(w[1]);
  }
  (void)elem;
  free(tau); free(ntau); free(p);
}

static void* worker(void* arg) {
  job_t* J = (job_t*)arg;
  for (uint64_t it = J->lo; it < J->hi; ++it) run_item(J, it);
  return NULL;
}

/* Neumaier's compensated summation (Neumaier 1974) */
typedef struct { double s, c; } nsum;
static void nsum_add(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}

static int run_estimator(const orc_scene* sc, int what, const double* theta, double sg,
                         uint64_t N, uint64_t seed, const double* v, const orc_opts* o,
                         double* out) {
  if (!sc || !theta || !out || !o) return -1;
  int n = sc->n;
  if (!(sg > 0) || !isfinite(sg) || N == 0 || N >= 0xFFFFFFFFull) return -1;
  if (o->s0 + N > 0xFFFFFFFFull) return -1;
  for (int j = 0; j < n; ++j) if (!isfinite(theta[j])) return -1;
  if (o->sampler < 0 || o->sampler > 3) return -1;
  if (o->hess_mix_n2 != 0 && o->hess_mix_n2 != 1) return -1;
  if (what == W_HVPL && per_element(o->sampler)) return -4;
  if (o->sampler == ORC_FR22 && what == W_HESS) return -4;
  int hess_kernel = (what == W_HESS || what == W_HVPL);
  int K = hess_kernel ? n * (n + 1) / 2 : n;
  int nout = what == W_HESS ? K : n;
  int A = o->antithetic ? 2 : 1;

  job_t J;
  memset(&J, 0, sizeof(J));
  J.sc = sc; J.what = what; J.n = n; J.K = K; J.sampler = o->sampler; J.A = A;
  J.mix_n2 = o->hess_mix_n2;
  J.nsh = what == W_HVP ? 2 : 1;
  J.theta = theta; J.sg = sg; J.N = N; J.seed = seed; J.s0 = o->s0; J.dbg = o->dbg_loss;

  double* u = NULL;
  if (what == W_HVP || what == W_HVPL) {
    if (!v) return -1;
    double vn = 0.0;
    for (int j = 0; j < n; ++j) {
      if (!isfinite(v[j])) return -1;
      vn += v[j] * v[j];
    }
    vn = sqrt(vn);
    if (vn == 0.0) {   /* H 0 = 0: no renders */
      for (int j = 0; j < n; ++j) out[j] = 0.0;
      return 0;
    }
    if (!(o->hvp_rel_step > 0)) return -1;
    J.vnorm = vn;
    J.h = o->hvp_rel_step * sg;
    u = (double*)malloc((size_t)n * sizeof(double));
    for (int j = 0; j < n; ++j) u[j] = v[j] / vn;
    J.u = u;
    J.v = v;
  }
  uint64_t items = per_element(o->sampler) ? (uint64_t)K * N : N;
  uint64_t per_item = per_element(o->sampler) ? 1 : (uint64_t)(what == W_HVPL ? n : K);
  J.contrib = (double*)malloc(items * per_item * sizeof(double));
  if (!J.contrib) { free(u); return -2; }
  tri_table tri = tri_make(n);
  J.T = &tri;

  int T = o->nthreads > 0 ? o->nthreads : 1;
  if ((uint64_t)T > items) T = (int)items;
  pthread_t* th = (pthread_t*)malloc((size_t)T * sizeof(pthread_t));
  job_t* jobs = (job_t*)malloc((size_t)T * sizeof(job_t));
  for (int t = 0; t < T; ++t) {
    jobs[t] = J;
    jobs[t].lo = items * (uint64_t)t / (uint64_t)T;
    jobs[t].hi = items * (uint64_t)(t + 1) / (uint64_t)T;
    if (T == 1) worker(&jobs[t]);
    else pthread_create(&th[t], NULL, worker, &jobs[t]);
  }
  if (T > 1) for (int t = 0; t < T; ++t) pthread_join(th[t], NULL);

  /* est_m = (1/(A N)) sum_s c_{s,m}, summed in sample order */
  double* est = (double*)malloc((size_t)nout * sizeof(double));
  for (int m = 0; m < nout; ++m) {
    nsum acc = {0.0, 0.0};
    for (uint64_t s = 0; s < N; ++s) {
      double x;
      if (per_element(o->sampler)) x = J.contrib[(uint64_t)m * N + s];
      else x = J.contrib[s * per_item + (uint64_t)m];
      nsum_add(&acc, x);
    }
    est[m] = (acc.s + acc.c) / ((double)A * (double)N);
  }
  if (what == W_HESS) {   /* mirror the upper triangle */
    for (int m = 0; m < K; ++m) {
      out[tri.i[m] * n + tri.j[m]] = est[m];
      out[tri.j[m] * n + tri.i[m]] = est[m];
    }
  } else {
    for (int m = 0; m < n; ++m) out[m] = est[m];
  }
  free(est); free(J.contrib); free(th); free(jobs); free(u);
  tri_free(&tri);
  return 0;
}

int orc_est_grad(const orc_scene* sc, const double* theta, double sigma, uint64_t N,
                 uint64_t seed, const orc_opts* o, double* g) {
  return run_estimator(sc, W_GRAD, theta, sigma, N, seed, NULL, o, g);
}
int orc_est_hessian(const orc_scene* sc, const double* theta, double sigma, uint64_t N,
                    uint64_t seed, const orc_opts* o, double* H) {
  return run_estimator(sc, W_HESS, theta, sigma, N, seed, NULL, o, H);
}
/* Section "Hessian-vector product": the HVP is the central difference of two
 * gradient estimators along v.  Read as Hv ~ |v| (g(theta + h u) - g(theta - h u))/(2h)
 * with u = v/|v|, h = c sigma, and the same draws (common random numbers) for
 * both shifts.  (The printed kernel form subtracts in the other order, which
 * under the convolution convention f(theta - tau) integrates to -Hv.) */
int orc_est_hvp(const orc_scene* sc, const double* theta, double sigma, uint64_t N,
                uint64_t seed, const double* v, const orc_opts* o, double* Hv) {
  return run_estimator(sc, W_HVP, theta, sigma, N, seed, v, o, Hv);
}
int orc_est_hvp_limit(const orc_scene* sc, const double* theta, double sigma, uint64_t N,
                      uint64_t seed, const double* v, const orc_opts* o, double* Hv) {
  return run_estimator(sc, W_HVPL, theta, sigma, N, seed, v, o, Hv);
}

/* ========================================================================= */
/* Smoothed loss (section "Background"): F(theta) = E f(theta - tau) over
 * Gaussian draws (the plain sampler's draws), antithetic pairs as set; the
 * mean is summed in draw order.  sigma = 0: the plain loss.                   */
/* ========================================================================= */
int orc_est_loss(const orc_scene* sc, const double* theta, double sigma, uint64_t N,
                 uint64_t seed, const orc_opts* o, double* F) {
  if (!sc || !theta || !F || !o) return -1;
  int n = sc->n;
  for (int j = 0; j < n; ++j) if (!isfinite(theta[j])) return -1;
  if (sigma == 0.0) {
    *F = orc_loss(sc, theta, seed, 0);
    return 0;
  }
  if (!(sigma > 0) || !isfinite(sigma) || N == 0 || N >= 0xFFFFFFFFull) return -1;
  int A = o->antithetic ? 2 : 1;
  double* tau = (double*)malloc((size_t)n * sizeof(double));
  double* p = (double*)malloc((size_t)n * sizeof(double));
  nsum acc = {0.0, 0.0};
  for (uint64_t s = 0; s < N; ++s) {
    int e;
    draw(0, n, sigma, seed, (uint32_t)s, ORC_GAUSS, 0, 0, tau, &e);
    for (int ai = 0; ai < A; ++ai) {
      double a = ai == 0 ? 1.0 : -1.0;
      for (int j = 0; j < n; ++j) p[j] = theta[j] - a * tau[j];
      nsum_add(&acc, orc_loss(sc, p, seed, (uint32_t)s));
    }
  }
  *F = (acc.s + acc.c) / ((double)A * (double)N);
  free(tau);
  free(p);
  return 0;
}

/* ========================================================================= */
/* Grey-box composition (appendix "Grey-box differentials"): gradient J^T g_y,
 * Hessian J^T H_y J, HVP J^T H_y J v, with the outer derivatives sampled.    */
/* ========================================================================= */
int orc_est_grad_greybox(const orc_scene* sc, const double* y, const double* J, int n_in,
                         double sigma, uint64_t N, uint64_t seed, const orc_opts* o, double* gx) {
  if (!sc || !J || !gx || n_in <= 0) return -1;
  int n = sc->n;
  double* gy = (double*)malloc((size_t)n * sizeof(double));
  int st = orc_est_grad(sc, y, sigma, N, seed, o, gy);
  if (!st)
    for (int a = 0; a < n_in; ++a) {
      double acc = 0.0;
      for (int i = 0; i < n; ++i) acc += J[(size_t)i * n_in + a] * gy[i];
      gx[a] = acc;
    }
  free(gy);
  return st;
}

int orc_est_hessian_greybox(const orc_scene* sc, const double* y, const double* J, int n_in,
                            double sigma, uint64_t N, uint64_t seed, const orc_opts* o,
                            double* Hx) {
  if (!sc || !J || !Hx || n_in <= 0) return -1;
  int n = sc->n;
  double* Hy = (double*)malloc((size_t)n * n * sizeof(double));
  int st = orc_est_hessian(sc, y, sigma, N, seed, o, Hy);
  if (!st)
    for (int a = 0; a < n_in; ++a)
      for (int b = 0; b < n_in; ++b) {
        double acc = 0.0;
        for (int i = 0; i < n; ++i)
          for (int k = 0; k < n; ++k)
            acc += J[(size_t)i * n_in + a] * Hy[(size_t)i * n + k] * J[(size_t)k * n_in + b];
        Hx[(size_t)a * n_in + b] = acc;
      }
  free(Hy);
  return st;
}

int orc_est_hvp_greybox(const orc_scene* sc, const double* y, const double* J, int n_in,
                        double sigma, uint64_t N, uint64_t seed, const double* vx,
                        const orc_opts* o, double* Hvx) {
  if (!sc || !J || !Hvx || !vx || n_in <= 0) return -1;
  int n = sc->n;
  double* vy = (double*)malloc((size_t)n * sizeof(double));
  double* hy = (double*)malloc((size_t)n * sizeof(double));
  for (int i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int a = 0; a < n_in; ++a) acc += J[(size_t)i * n_in + a] * vx[a];
    vy[i] = acc;
  }
  int st = orc_est_hvp(sc, y, sigma, N, seed, vy, o, hy);
  if (!st)
    for (int a = 0; a < n_in; ++a) {
      double acc = 0.0;
      for (int i = 0; i < n; ++i) acc += J[(size_t)i * n_in + a] * hy[i];
      Hvx[a] = acc;
    }
  free(vy);
  free(hy);
  return st;
}

/* ========================================================================= */
/* Symmetric eigen-decomposition: cyclic Jacobi (Jacobi 1846; Golub & Van Loan,
 * "Matrix Computations", cyclic Jacobi).  evecs column k belongs to evals[k]. */
/* ========================================================================= */
int orc_jacobi_eig(int n, const double* A, double* evals, double* evecs) {
  double* a = copy_d(A, (size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) evecs[i * n + j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a[i * n + j] * a[i * n + j];
        if (i != j) off += a[i * n + j] * a[i * n + j];
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = a[p * n + q];
        if (apq == 0.0) continue;
        double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {   /* A <- A J (columns p, q) */
          double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   /* A <- J^T A (rows p, q) */
          double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {   /* V <- V J */
          double vkp = evecs[k * n + p], vkq = evecs[k * n + q];
          evecs[k * n + p] = c * vkp - s * vkq;
          evecs[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) evals[i] = a[i * n + i];
  free(a);
  return 0;
}

/* ========================================================================= */
/* One Newton-CG step (section "Previous Work": Newton conjugate gradient with
 * the step length alpha = -g^T v / v^T H v, Fletcher-Reeves beta, and the trust
 * truncation alpha = min(alpha, Delta/|v|)).  Reading: the inner CG runs at the
 * fixed outer point theta_t (truncated Newton) with the same draws for every
 * product; a truncated or negative-curvature step ends the inner loop.        */
/* ========================================================================= */
static double vdot(int n, const double* a, const double* b) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

int orc_newton_cg_step(const orc_scene* sc, double* theta, double sigma, uint64_t N,
                       uint64_t seed, const orc_ncg_opts* no, const orc_opts* o,
                       orc_ncg_report* rep) {
  if (!sc || !theta || !no || !o) return -1;
  if (!(no->trust_radius > 0)) return -1;
  int n = sc->n;
  double* g = (double*)calloc((size_t)n, sizeof(double));
  double* d = (double*)calloc((size_t)n, sizeof(double));
  double* r = (double*)calloc((size_t)n, sizeof(double));
  double* p = (double*)calloc((size_t)n, sizeof(double));
  double* Hp = (double*)calloc((size_t)n, sizeof(double));
  orc_ncg_report R;
  memset(&R, 0, sizeof(R));
  int st = orc_est_grad(sc, theta, sigma, N, seed, o, g);
  if (st) goto done;
  R.g_norm = sqrt(vdot(n, g, g));
  if (no->use_full_hessian) {
    /* modified Newton: H = V L V^T, L <- max(|L|, floor), d = -V L^-1 V^T g,
     * then scaled back into the trust radius */
    double* H = (double*)malloc((size_t)n * n * sizeof(double));
    double* ev = (double*)malloc((size_t)n * sizeof(double));
    double* V = (double*)malloc((size_t)n * n * sizeof(double));
    st = orc_est_hessian(sc, theta, sigma, N, seed, o, H);
    if (!st) {
      orc_jacobi_eig(n, H, ev, V);
      for (int k = 0; k < n; ++k) {
        double lam = fabs(ev[k]);
        if (lam < no->eig_floor) lam = no->eig_floor;
        if (lam == 0.0) continue;   /* zero curvature and no floor: no step along it */
        double proj = 0.0;
        for (int i = 0; i < n; ++i) proj += V[i * n + k] * g[i];
        for (int i = 0; i < n; ++i) d[i] -= V[i * n + k] * proj / lam;
      }
      double dn = sqrt(vdot(n, d, d));
      if (dn > no->trust_radius) {
        for (int i = 0; i < n; ++i) d[i] *= no->trust_radius / dn;
        R.hit_trust = 1;
      }
      R.iters_done = 1;
    }
    free(H); free(ev); free(V);
  } else {
    for (int i = 0; i < n; ++i) { r[i] = -g[i]; p[i] = r[i]; }
    double rr = vdot(n, r, r);
    for (int k = 0; k < no->cg_iters; ++k) {
      double pn = sqrt(vdot(n, p, p));
      if (pn == 0.0) break;
      st = no->hvp_limit ? orc_est_hvp_limit(sc, theta, sigma, N, seed, p, o, Hp)
                         : orc_est_hvp(sc, theta, sigma, N, seed, p, o, Hp);
      if (st) goto done;
      R.iters_done = k + 1;
      double curv = vdot(n, p, Hp);
      if (no->modified) {
        /* reading of the paper's "Hessian modification and truncation to a
         * trust region" inside CG: a non-positive curvature is replaced by its
         * magnitude (floored), alpha = min(alpha, Delta/|v|), and CG goes on */
        double kappa = fabs(curv);
        if (curv <= 0.0) R.neg_curv = 1;
        if (kappa < no->eig_floor * pn * pn) kappa = no->eig_floor * pn * pn;
        if (kappa == 0.0) break;
        double alpha = rr / kappa;
        if (alpha > no->trust_radius / pn) {
          alpha = no->trust_radius / pn;
          R.hit_trust = 1;
        }
        for (int i = 0; i < n; ++i) d[i] += alpha * p[i];
        for (int i = 0; i < n; ++i) r[i] -= alpha * Hp[i];
        double rr_new = vdot(n, r, r);
        if (sqrt(rr_new) <= 1e-10 * R.g_norm) break;
        double beta = rr_new / rr;
        for (int i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        continue;
      }
      if (curv <= 0.0) {
        double a = no->trust_radius / pn;
        for (int i = 0; i < n; ++i) d[i] += a * p[i];
        R.neg_curv = 1;
        break;
      }
      double alpha = rr / curv;
      if (alpha > no->trust_radius / pn) {
        alpha = no->trust_radius / pn;
        for (int i = 0; i < n; ++i) d[i] += alpha * p[i];
        R.hit_trust = 1;
        break;
      }
      for (int i = 0; i < n; ++i) d[i] += alpha * p[i];
      for (int i = 0; i < n; ++i) r[i] -= alpha * Hp[i];
      double rr_new = vdot(n, r, r);
      if (sqrt(rr_new) <= 1e-10 * R.g_norm) break;
      double beta = rr_new / rr;
      for (int i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
      rr = rr_new;
    }
  }
  for (int i = 0; i < n; ++i) theta[i] += d[i];
  R.step_norm = sqrt(vdot(n, d, d));
done:
  if (rep) *rep = R;
  free(g); free(d); free(r); free(p); free(Hp);
  return st;
}

/* ========================================================================= */
/* Optimiser loop (appendix "Hyperparameters"; reading of "recompute" and of
 * the line search stated in orc.h).                                          */
/* ========================================================================= */
int orc_optimize(const orc_scene* sc, double* theta, uint64_t N, uint64_t seed,
                 const orc_optim_opts* oo, const orc_opts* o, double* trace) {
  if (!sc || !theta || !oo || !o) return -1;
  if (oo->iters < 1 || oo->recompute < 1 || oo->ls_iters < 0) return -1;
  if (!(oo->sigma_start > 0) || !(oo->sigma_end > 0)) return -1;
  if (oo->method < 0 || oo->method > 2) return -1;
  if (oo->ls_iters > 0 && oo->N_loss == 0) return -1;
  int n = sc->n;
  double* d = (double*)malloc((size_t)n * sizeof(double));
  double* trial = (double*)malloc((size_t)n * sizeof(double));
  double alpha_keep = 1.0;
  int st = 0;
  for (int t = 0; t < oo->iters; ++t) {
    double sg = oo->iters > 1
                    ? oo->sigma_start + (oo->sigma_end - oo->sigma_start) * t / (double)(oo->iters - 1)
                    : oo->sigma_start;
    uint64_t sd = seed + (uint64_t)t;
    if (oo->method == ORC_OPT_GD) {
      st = orc_est_grad(sc, theta, sg, N, sd, o, d);
      if (st) break;
      for (int i = 0; i < n; ++i) d[i] = -oo->lr * d[i];
    } else {
      orc_ncg_opts no = oo->ncg;
      no.use_full_hessian = oo->method == ORC_OPT_NEWTON_FULL;
      for (int i = 0; i < n; ++i) trial[i] = theta[i];
      st = orc_newton_cg_step(sc, trial, sg, N, sd, &no, o, NULL);
      if (st) break;
      for (int i = 0; i < n; ++i) d[i] = trial[i] - theta[i];
    }
    double alpha = 1.0;
    if (oo->ls_iters > 0) {
      if (t % oo->recompute == 0) {
        double F0, F1;
        st = orc_est_loss(sc, theta, sg, oo->N_loss, sd, o, &F0);
        if (st) break;
        alpha = 1.0;
        int ok = 0;
        for (int k = 0; k < oo->ls_iters; ++k) {
          for (int i = 0; i < n; ++i) trial[i] = theta[i] + alpha * d[i];
          st = orc_est_loss(sc, trial, sg, oo->N_loss, sd, o, &F1);
          if (st) break;
          if (F1 <= F0 - oo->ls_tol * fabs(F0)) { ok = 1; break; }
          alpha *= 0.5;
        }
        if (st) break;
        if (!ok) alpha = 0.0;   /* no decrease found: stay */
        alpha_keep = alpha;
      } else {
        alpha = alpha_keep;
      }
    }
    double sn = 0.0;
    for (int i = 0; i < n; ++i) {
      theta[i] += alpha * d[i];
      sn += (alpha * d[i]) * (alpha * d[i]);
    }
    if (trace) {
      double Fs = 0.0, f = 0.0;
      uint64_t nl = oo->N_loss > 0 ? oo->N_loss : N;
      st = orc_est_loss(sc, theta, sg, nl, sd, o, &Fs);
      if (!st) st = orc_est_loss(sc, theta, 0.0, 1, sd, o, &f);
      if (st) break;
      double* row = trace + 5 * (size_t)t;
      row[0] = sg; row[1] = alpha; row[2] = sqrt(sn); row[3] = Fs; row[4] = f;
    }
  }
  free(d);
  free(trial);
  return st;
}
