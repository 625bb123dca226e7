/*
 * gs_oracle.c -- FP64 CPU oracle of the differentiable Gaussian-splatting
 * rasterizer that the joint pose + Gaussian optimisation runs forward and
 * backward in every step (paper section 4.3; the rasterizer is the one of
 * the 3DGS codebase the paper builds on, section 5, so its compositing model
 * is the standard EWA-splatting one and is restated here from first
 * principles).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this file.  The product path (the
 * HIP library) never calls it, and the two share no code, headers or tables.
 *
 * What this computes is the plain definition, with no acceleration beyond a
 * conservative bounding-box pre-test:
 *   * every Gaussian is projected on its own (EWA: Sigma2 = J W Sigma W^T J^T
 *     + eps I).  With the screen-space filter of multi-scale training
 *     (section 4.3 cites Mip-Splatting for it), eps I is the covariance of a
 *     Gaussian low-pass filter convolved with the splat, and the opacity is
 *     scaled by rho = sqrt(det(Sigma2 - eps I) / det Sigma2) so that the
 *     splat's integral o rho 2 pi sqrt(det Sigma2) does not depend on eps;
 *   * the visible Gaussians are put in (depth, index) order once;
 *   * every pixel walks ALL of them front to back: alpha = min(alpha_max,
 *     o * exp(-d^T Sigma2^-1 d / 2)); an alpha below alpha_min is skipped;
 *     if the transmittance after a Gaussian would fall below t_min the pixel
 *     stops without it; otherwise colour, depth and transmittance update.
 *   * gradients are the analytic adjoint: per pixel over the recorded list
 *     with explicit suffix sums, then per Gaussian through conic -> Sigma2 ->
 *     (J, W Sigma W^T) -> (p, R) -> (mean, t), Sigma -> (log-scales,
 *     quaternion through its normalisation), colour -> SH and -> mean via the
 *     view direction, opacity -> logit.  The camera pose receives gradient
 *     through the projected position and the covariance only, never through
 *     the SH view direction (section 4.3, pose optimisation).
 *
 * Arithmetic is IEEE double throughout; threads split pixel rows and every
 * cross-thread sum is taken in a fixed order, so results are deterministic.
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_THREADS 256

typedef struct {
  double R[9]; /* world -> camera rotation, row-major */
  double t[3]; /* world -> camera translation */
  double fx, fy, cx, cy;
  int32_t width, height;
  double near_plane;
  double bg[3];
  double eps2d;     /* dilation added to the 2D covariance */
  double alpha_max; /* opacity clamp */
  double alpha_min; /* smallest alpha that is composited */
  double t_min;     /* transmittance cutoff */
  double guard;     /* guard band factor of the Jacobian clamp */
  int32_t mip_filter; /* 1: eps2d is a screen-space filter with opacity compensation */
} orc_cam;

typedef struct {
  int64_t n;
  int32_t sh_degree;
  const double *means;          /* [3][n] */
  const double *log_scales;     /* [3][n] */
  const double *quats;          /* [4][n]  (w, x, y, z), need not be unit */
  const double *opacity_logits; /* [n] */
  const double *sh;             /* [(deg+1)^2][3][n] */
} orc_gauss;

typedef struct {
  double *mean2d;   /* [2][n] */
  double *depth;    /* [n] */
  double *conic;    /* [3][n]  (A, B, C) of Sigma2^-1 = [[A, B], [B, C]] */
  double *cov2d;    /* [3][n]  (a, b, c) of Sigma2 = [[a, b], [b, c]] */
  double *opacity;  /* [n] */
  double *rgb;      /* [3][n] */
  double *radius;   /* [n]  sqrt(2 ln(o / alpha_min) lambda_max), unrounded */
  double *half;     /* [2][n] half-extents of the support ellipse's bounding box */
  int32_t *visible; /* [n]  1 if the Gaussian can contribute anywhere */
  int32_t *clamped; /* [n]  bit c set if colour channel c was clamped at 0 */
} orc_proj;

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics up to degree 3 on a unit direction (x, y, z).     */
/* Normalised so that the integral of Y_i Y_j over the sphere is delta_ij;    */
/* signs follow the Condon-Shortley phase used by 3DGS colour models.         */
/* ------------------------------------------------------------------------ */
static void sh_consts(double c[16]) {
  const double sp = sqrt(M_PI);
  c[0] = 1.0 / (2.0 * sp);
  c[1] = -sqrt(3.0) / (2.0 * sp);
  c[2] = sqrt(3.0) / (2.0 * sp);
  c[3] = -sqrt(3.0) / (2.0 * sp);
  c[4] = sqrt(15.0) / (2.0 * sp);
  c[5] = -sqrt(15.0) / (2.0 * sp);
  c[6] = sqrt(5.0) / (4.0 * sp);
  c[7] = -sqrt(15.0) / (2.0 * sp);
  c[8] = sqrt(15.0) / (4.0 * sp);
  c[9] = -sqrt(35.0 / 2.0) / (4.0 * sp);
  c[10] = sqrt(105.0) / (2.0 * sp);
  c[11] = -sqrt(21.0 / 2.0) / (4.0 * sp);
  c[12] = sqrt(7.0) / (4.0 * sp);
  c[13] = -sqrt(21.0 / 2.0) / (4.0 * sp);
  c[14] = sqrt(105.0) / (4.0 * sp);
  c[15] = -sqrt(35.0 / 2.0) / (4.0 * sp);
}

/* Y[k] and its gradient dY[k][0..2] with respect to (x, y, z) treated as
 * independent variables (the caller projects onto the sphere's tangent). */
static void sh_eval(int deg, const double d[3], double Y[16], double dY[16][3]) {
  double c[16];
  sh_consts(c);
  const double x = d[0], y = d[1], z = d[2];
  const int nb = (deg + 1) * (deg + 1);
  double P[16], G[16][3];
  memset(G, 0, sizeof(G));
  P[0] = 1.0;
  if (deg >= 1) {
    P[1] = y; G[1][1] = 1.0;
    P[2] = z; G[2][2] = 1.0;
    P[3] = x; G[3][0] = 1.0;
  }
  if (deg >= 2) {
    P[4] = x * y; G[4][0] = y; G[4][1] = x;
    P[5] = y * z; G[5][1] = z; G[5][2] = y;
    P[6] = 2.0 * z * z - x * x - y * y; G[6][0] = -2.0 * x; G[6][1] = -2.0 * y; G[6][2] = 4.0 * z;
    P[7] = x * z; G[7][0] = z; G[7][2] = x;
    P[8] = x * x - y * y; G[8][0] = 2.0 * x; G[8][1] = -2.0 * y;
  }
  if (deg >= 3) {
    P[9] = y * (3.0 * x * x - y * y);
    G[9][0] = 6.0 * x * y; G[9][1] = 3.0 * x * x - 3.0 * y * y;
    P[10] = x * y * z;
    G[10][0] = y * z; G[10][1] = x * z; G[10][2] = x * y;
    P[11] = y * (4.0 * z * z - x * x - y * y);
    G[11][0] = -2.0 * x * y; G[11][1] = 4.0 * z * z - x * x - 3.0 * y * y; G[11][2] = 8.0 * y * z;
    P[12] = z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    G[12][0] = -6.0 * x * z; G[12][1] = -6.0 * y * z; G[12][2] = 6.0 * z * z - 3.0 * x * x - 3.0 * y * y;
    P[13] = x * (4.0 * z * z - x * x - y * y);
    G[13][0] = 4.0 * z * z - 3.0 * x * x - y * y; G[13][1] = -2.0 * x * y; G[13][2] = 8.0 * x * z;
    P[14] = z * (x * x - y * y);
    G[14][0] = 2.0 * x * z; G[14][1] = -2.0 * y * z; G[14][2] = x * x - y * y;
    P[15] = x * (x * x - 3.0 * y * y);
    G[15][0] = 3.0 * x * x - 3.0 * y * y; G[15][1] = -6.0 * x * y;
  }
  for (int k = 0; k < nb; ++k) {
    Y[k] = c[k] * P[k];
    if (dY)
      for (int a = 0; a < 3; ++a) dY[k][a] = c[k] * G[k][a];
  }
}

/* Exposed for the orthonormality pin. */
void orc_sh_basis(int deg, const double *dir, double *out16) {
  double Y[16];
  sh_eval(deg, dir, Y, NULL);
  for (int k = 0; k < (deg + 1) * (deg + 1); ++k) out16[k] = Y[k];
}

/* Rotation matrix (row-major) of a unit quaternion (w, x, y, z). */
static void quat_to_rot(const double q[4], double Rq[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  Rq[0] = 1.0 - 2.0 * (y * y + z * z);
  Rq[1] = 2.0 * (x * y - w * z);
  Rq[2] = 2.0 * (x * z + w * y);
  Rq[3] = 2.0 * (x * y + w * z);
  Rq[4] = 1.0 - 2.0 * (x * x + z * z);
  Rq[5] = 2.0 * (y * z - w * x);
  Rq[6] = 2.0 * (x * z - w * y);
  Rq[7] = 2.0 * (y * z + w * x);
  Rq[8] = 1.0 - 2.0 * (x * x + y * y);
}

void orc_quat_to_rot(const double *q, double *R9) {
  double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double u[4] = {q[0] / n, q[1] / n, q[2] / n, q[3] / n};
  quat_to_rot(u, R9);
}

/* Gradient of sum_ij G_ij Rq_ij with respect to the unit quaternion. */
static void quat_to_rot_vjp(const double q[4], const double G[9], double gq[4]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  /* d Rq_ij / d(w, x, y, z), entry by entry */
  gq[0] = G[1] * (-2 * z) + G[2] * (2 * y) + G[3] * (2 * z) + G[5] * (-2 * x) + G[6] * (-2 * y) +
          G[7] * (2 * x);
  gq[1] = G[1] * (2 * y) + G[2] * (2 * z) + G[3] * (2 * y) + G[4] * (-4 * x) + G[5] * (-2 * w) +
          G[6] * (2 * z) + G[7] * (2 * w) + G[8] * (-4 * x);
  gq[2] = G[0] * (-4 * y) + G[1] * (2 * x) + G[2] * (2 * w) + G[3] * (2 * x) + G[5] * (2 * z) +
          G[6] * (-2 * w) + G[7] * (2 * z) + G[8] * (-4 * y);
  gq[3] = G[0] * (-4 * z) + G[1] * (-2 * w) + G[2] * (2 * x) + G[3] * (2 * w) + G[4] * (-4 * z) +
          G[5] * (2 * y) + G[6] * (2 * x) + G[7] * (2 * y);
}

/* Everything the forward of one Gaussian produces, kept for its backward. */
typedef struct {
  int visible;
  double p[3], z, xc, yc;
  int clx, cly; /* Jacobian clamp active on x / y */
  double qn[4], qnorm, Rq[9], s[3], M[9], Sig[9], V[9], J[6];
  double a, b, c, det, A, B, C;
  double a0, c0, det0, rho, osig; /* unfiltered covariance, its determinant, compensation, sigmoid */
  double mx, my, o, lmax, rarg, hx, hy;
  double dir[3], dnorm, dhat[3], val[3], rgb[3];
  int clamped;
} gfwd;

static void mat3_mul(const double *X, const double *Y, double *Z) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += X[3 * i + k] * Y[3 * k + j];
      Z[3 * i + j] = s;
    }
}
static void mat3_mul_bt(const double *X, const double *Y, double *Z) { /* X Y^T */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += X[3 * i + k] * Y[3 * j + k];
      Z[3 * i + j] = s;
    }
}
static void mat3_mul_at(const double *X, const double *Y, double *Z) { /* X^T Y */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += X[3 * k + i] * Y[3 * k + j];
      Z[3 * i + j] = s;
    }
}

static void project_one(const orc_cam *cam, const orc_gauss *g, int64_t i, gfwd *f) {
  const int64_t n = g->n;
  memset(f, 0, sizeof(*f));
  const double mu[3] = {g->means[i], g->means[n + i], g->means[2 * n + i]};
  const double *R = cam->R;
  for (int r = 0; r < 3; ++r) f->p[r] = R[3 * r] * mu[0] + R[3 * r + 1] * mu[1] + R[3 * r + 2] * mu[2] + cam->t[r];
  f->z = f->p[2];
  if (!(f->z > cam->near_plane)) return;

  /* Jacobian of the perspective map, with the 3DGS guard band */
  const double z = f->z;
  const double limx = cam->guard * 0.5 * cam->width / cam->fx;
  const double limy = cam->guard * 0.5 * cam->height / cam->fy;
  const double tx = f->p[0] / z, ty = f->p[1] / z;
  f->clx = (tx < -limx || tx > limx);
  f->cly = (ty < -limy || ty > limy);
  f->xc = f->clx ? (tx < 0 ? -limx : limx) * z : f->p[0];
  f->yc = f->cly ? (ty < 0 ? -limy : limy) * z : f->p[1];
  f->J[0] = cam->fx / z; f->J[1] = 0.0; f->J[2] = -cam->fx * f->xc / (z * z);
  f->J[3] = 0.0; f->J[4] = cam->fy / z; f->J[5] = -cam->fy * f->yc / (z * z);

  /* 3D covariance Sigma = Rq S S^T Rq^T */
  const double q[4] = {g->quats[i], g->quats[n + i], g->quats[2 * n + i], g->quats[3 * n + i]};
  f->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) f->qn[k] = q[k] / f->qnorm;
  quat_to_rot(f->qn, f->Rq);
  for (int k = 0; k < 3; ++k) f->s[k] = exp(g->log_scales[k * n + i]);
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc) f->M[3 * r + cc] = f->Rq[3 * r + cc] * f->s[cc];
  mat3_mul_bt(f->M, f->M, f->Sig);
  /* camera-frame covariance V = R Sigma R^T */
  double RS[9];
  mat3_mul(R, f->Sig, RS);
  mat3_mul_bt(RS, R, f->V);
  /* Sigma2 = J V J^T + eps I */
  double JV[6];
  for (int r = 0; r < 2; ++r)
    for (int cc = 0; cc < 3; ++cc)
      JV[3 * r + cc] = f->J[3 * r] * f->V[cc] + f->J[3 * r + 1] * f->V[3 + cc] + f->J[3 * r + 2] * f->V[6 + cc];
  double S2[4];
  for (int r = 0; r < 2; ++r)
    for (int cc = 0; cc < 2; ++cc)
      S2[2 * r + cc] = JV[3 * r] * f->J[3 * cc] + JV[3 * r + 1] * f->J[3 * cc + 1] + JV[3 * r + 2] * f->J[3 * cc + 2];
  f->a0 = S2[0];
  f->c0 = S2[3];
  f->a = S2[0] + cam->eps2d;
  f->b = 0.5 * (S2[1] + S2[2]);
  f->c = S2[3] + cam->eps2d;
  f->det = f->a * f->c - f->b * f->b;
  f->det0 = f->a0 * f->c0 - f->b * f->b;
  if (!(f->det > 0.0)) return;
  f->A = f->c / f->det;
  f->B = -f->b / f->det;
  f->C = f->a / f->det;

  f->mx = cam->fx * f->p[0] / z + cam->cx;
  f->my = cam->fy * f->p[1] / z + cam->cy;

  const double al = g->opacity_logits[i];
  f->osig = 1.0 / (1.0 + exp(-al));
  f->rho = cam->mip_filter ? sqrt(fmax(f->det0, 0.0) / f->det) : 1.0;
  f->o = f->osig * f->rho;
  if (!(f->o >= cam->alpha_min)) return;
  const double h = 0.5 * (f->a - f->c);
  f->lmax = 0.5 * (f->a + f->c) + sqrt(h * h + f->b * f->b);
  f->rarg = sqrt(2.0 * log(f->o / cam->alpha_min) * f->lmax);
  /* alpha >= alpha_min  <=>  d^T Sigma2^-1 d <= qmax; that ellipse's
     axis-aligned bounding box has half-extents sqrt(qmax Sigma2_xx), ... */
  f->hx = sqrt(2.0 * log(f->o / cam->alpha_min) * f->a);
  f->hy = sqrt(2.0 * log(f->o / cam->alpha_min) * f->c);

  /* view-dependent colour from SH, view direction from the camera centre */
  const double Cw[3] = {-(R[0] * cam->t[0] + R[3] * cam->t[1] + R[6] * cam->t[2]),
                        -(R[1] * cam->t[0] + R[4] * cam->t[1] + R[7] * cam->t[2]),
                        -(R[2] * cam->t[0] + R[5] * cam->t[1] + R[8] * cam->t[2])};
  for (int k = 0; k < 3; ++k) f->dir[k] = mu[k] - Cw[k];
  f->dnorm = sqrt(f->dir[0] * f->dir[0] + f->dir[1] * f->dir[1] + f->dir[2] * f->dir[2]);
  for (int k = 0; k < 3; ++k) f->dhat[k] = f->dir[k] / f->dnorm;
  double Y[16];
  sh_eval(g->sh_degree, f->dhat, Y, NULL);
  const int nb = (g->sh_degree + 1) * (g->sh_degree + 1);
  for (int ch = 0; ch < 3; ++ch) {
    double v = 0.5;
    for (int k = 0; k < nb; ++k) v += g->sh[(k * 3 + ch) * n + i] * Y[k];
    f->val[ch] = v;
    if (v > 0.0) {
      f->rgb[ch] = v;
    } else {
      f->rgb[ch] = 0.0;
      f->clamped |= 1 << ch;
    }
  }
  f->visible = 1;
}

/* ------------------------------------------------------------------------ */
/* Projection (forward), all Gaussians.                                       */
/* ------------------------------------------------------------------------ */
void orc_project(const orc_cam *cam, const orc_gauss *g, orc_proj *out) {
  const int64_t n = g->n;
  for (int64_t i = 0; i < n; ++i) {
    gfwd f;
    project_one(cam, g, i, &f);
    out->visible[i] = f.visible;
    out->mean2d[i] = f.mx;
    out->mean2d[n + i] = f.my;
    out->depth[i] = f.z;
    out->conic[i] = f.A;
    out->conic[n + i] = f.B;
    out->conic[2 * n + i] = f.C;
    out->cov2d[i] = f.a;
    out->cov2d[n + i] = f.b;
    out->cov2d[2 * n + i] = f.c;
    out->opacity[i] = f.o;
    for (int ch = 0; ch < 3; ++ch) out->rgb[ch * n + i] = f.rgb[ch];
    out->radius[i] = f.rarg;
    out->half[i] = f.hx;
    out->half[n + i] = f.hy;
    out->clamped[i] = f.clamped;
  }
}

/* ------------------------------------------------------------------------ */
/* Per-pixel compositing over a crop [x0, x0+cw) x [y0, y0+ch).               */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_cam *cam;
  const orc_proj *pr;
  int64_t n;
  const int64_t *order; /* candidates in (depth, index) order */
  int64_t n_order;
  int32_t x0, y0, cw, ch;
  double flag_rel;
  /* forward outputs (crop-sized, may be NULL) */
  double *image, *depth, *alpha, *final_t;
  int32_t *n_contrib, *n_support, *flags;
  /* backward */
  const double *g_image, *g_depth, *g_alpha;
  double *g2d_threads; /* [nthreads][n_order][10] */
  int nthreads;
  int rows_per;
} render_job;

typedef struct {
  render_job *job;
  int tid;
} render_task;

static int cmp_depth_index(const void *pa, const void *pb, void *ctx);

/* Evaluate Gaussian k of the list at pixel (u, v). */
static inline void eval_pair(const orc_proj *pr, int64_t n, int64_t i, double u, double v, double *dx, double *dy,
                             double *sexp, double *raw) {
  const double mx = pr->mean2d[i], my = pr->mean2d[n + i];
  const double A = pr->conic[i], B = pr->conic[n + i], C = pr->conic[2 * n + i];
  *dx = u - mx;
  *dy = v - my;
  const double s = -0.5 * (A * (*dx) * (*dx) + C * (*dy) * (*dy)) - B * (*dx) * (*dy);
  *sexp = exp(s);
  *raw = pr->opacity[i] * (*sexp);
}

static void *render_fwd_worker(void *arg) {
  render_task *task = (render_task *)arg;
  render_job *jb = task->job;
  const orc_cam *cam = jb->cam;
  const orc_proj *pr = jb->pr;
  const int64_t n = jb->n;
  const int r0 = task->tid * jb->rows_per;
  const int r1 = (r0 + jb->rows_per < jb->ch) ? r0 + jb->rows_per : jb->ch;
  const double fr = jb->flag_rel;
  for (int ry = r0; ry < r1; ++ry) {
    for (int rx = 0; rx < jb->cw; ++rx) {
      const double u = jb->x0 + rx, v = jb->y0 + ry;
      double T = 1.0, col[3] = {0, 0, 0}, D = 0.0;
      int ncomp = 0, nsup = 0, flag = 0;
      int64_t prev = -1; /* previous entry with alpha >= alpha_min */
      for (int64_t k = 0; k < jb->n_order; ++k) {
        const int64_t i = jb->order[k];
        const double rb = pr->radius[i] + 1.0;
        if (fabs(u - pr->mean2d[i]) > rb || fabs(v - pr->mean2d[n + i]) > rb) continue; /* pure speed-up */
        double dx, dy, e, raw;
        eval_pair(pr, n, i, u, v, &dx, &dy, &e, &raw);
        if (fabs(raw - cam->alpha_min) <= fr * cam->alpha_min) flag |= 1;
        if (raw >= cam->alpha_min * (1.0 - fr) && fabs(raw - cam->alpha_max) <= fr * cam->alpha_max) flag |= 2;
        const double alpha = raw < cam->alpha_max ? raw : cam->alpha_max;
        if (alpha < cam->alpha_min) continue;
        ++nsup;
        /* An implementation that orders by the binary32 rounding of the depth
           (ties by index) differs from (depth, index) order only where two
           roundings tie and the index order runs against the depth order. */
        if (prev >= 0 && (float)pr->depth[prev] == (float)pr->depth[i] && prev > i) flag |= 8;
        prev = i;
        const double Tn = T * (1.0 - alpha);
        if (fabs(Tn - cam->t_min) <= fr * cam->t_min) flag |= 4;
        if (Tn < cam->t_min) break;
        const double z = pr->depth[i];
        const double w = alpha * T;
        for (int c = 0; c < 3; ++c) col[c] += pr->rgb[c * n + i] * w;
        D += z * w;
        T = Tn;
        ++ncomp;
      }
      const int64_t o = (int64_t)ry * jb->cw + rx;
      const int64_t np = (int64_t)jb->cw * jb->ch;
      if (jb->image)
        for (int c = 0; c < 3; ++c) jb->image[c * np + o] = col[c] + T * cam->bg[c];
      if (jb->depth) jb->depth[o] = D;
      if (jb->alpha) jb->alpha[o] = 1.0 - T;
      if (jb->final_t) jb->final_t[o] = T;
      if (jb->n_contrib) jb->n_contrib[o] = ncomp;
      if (jb->n_support) jb->n_support[o] = nsup;
      if (jb->flags) jb->flags[o] = flag;
    }
  }
  return NULL;
}

/* Backward of the compositing at each pixel: first the list is recorded
 * front to back exactly as in the forward, then the suffix sums are formed
 * explicitly back to front and each entry's adjoint is evaluated. */
typedef struct {
  int64_t k; /* position in the candidate order */
  double dx, dy, e, raw, alpha, T;
} rec_entry;

static void *render_bwd_worker(void *arg) {
  render_task *task = (render_task *)arg;
  render_job *jb = task->job;
  const orc_cam *cam = jb->cam;
  const orc_proj *pr = jb->pr;
  const int64_t n = jb->n;
  double *g2d = jb->g2d_threads + (int64_t)task->tid * jb->n_order * 10;
  const int r0 = task->tid * jb->rows_per;
  const int r1 = (r0 + jb->rows_per < jb->ch) ? r0 + jb->rows_per : jb->ch;
  const int64_t np = (int64_t)jb->cw * jb->ch;
  rec_entry *list = (rec_entry *)malloc(sizeof(rec_entry) * (size_t)(jb->n_order > 0 ? jb->n_order : 1));
  for (int ry = r0; ry < r1; ++ry) {
    for (int rx = 0; rx < jb->cw; ++rx) {
      const double u = jb->x0 + rx, v = jb->y0 + ry;
      const int64_t o = (int64_t)ry * jb->cw + rx;
      int64_t L = 0;
      double T = 1.0;
      for (int64_t k = 0; k < jb->n_order; ++k) {
        const int64_t i = jb->order[k];
        const double rb = pr->radius[i] + 1.0;
        if (fabs(u - pr->mean2d[i]) > rb || fabs(v - pr->mean2d[n + i]) > rb) continue;
        double dx, dy, e, raw;
        eval_pair(pr, n, i, u, v, &dx, &dy, &e, &raw);
        const double alpha = raw < cam->alpha_max ? raw : cam->alpha_max;
        if (alpha < cam->alpha_min) continue;
        const double Tn = T * (1.0 - alpha);
        if (Tn < cam->t_min) break;
        rec_entry *r = &list[L++];
        r->k = k; r->dx = dx; r->dy = dy; r->e = e; r->raw = raw; r->alpha = alpha; r->T = T;
        T = Tn;
      }
      const double Tf = T;
      const double GC[3] = {jb->g_image ? jb->g_image[o] : 0.0, jb->g_image ? jb->g_image[np + o] : 0.0,
                            jb->g_image ? jb->g_image[2 * np + o] : 0.0};
      const double GD = jb->g_depth ? jb->g_depth[o] : 0.0;
      const double GA = jb->g_alpha ? jb->g_alpha[o] : 0.0;
      /* suffix sums S_k = sum_{j>k} c_j w_j + T_final bg, SD_k = sum_{j>k} z_j w_j */
      double S[3] = {Tf * cam->bg[0], Tf * cam->bg[1], Tf * cam->bg[2]}, SD = 0.0;
      for (int64_t e = L - 1; e >= 0; --e) {
        const rec_entry *r = &list[e];
        const int64_t i = jb->order[r->k];
        const double w = r->alpha * r->T;
        const double z = pr->depth[i];
        const double c3[3] = {pr->rgb[i], pr->rgb[n + i], pr->rgb[2 * n + i]};
        double *gg = g2d + r->k * 10;
        for (int c = 0; c < 3; ++c) gg[6 + c] += GC[c] * w;
        gg[9] += GD * w;
        const double inv = 1.0 / (1.0 - r->alpha);
        double ga = GA * Tf * inv + GD * (z * r->T - SD * inv);
        for (int c = 0; c < 3; ++c) ga += GC[c] * (c3[c] * r->T - S[c] * inv);
        if (r->raw < cam->alpha_max) {
          /* alpha = o exp(s): d/do = exp(s), d/ds = alpha */
          const double A = pr->conic[i], B = pr->conic[n + i], C = pr->conic[2 * n + i];
          const double gs = ga * r->raw;
          gg[5] += ga * r->e;
          gg[2] += gs * (-0.5 * r->dx * r->dx);
          gg[3] += gs * (-r->dx * r->dy);
          gg[4] += gs * (-0.5 * r->dy * r->dy);
          gg[0] += gs * (A * r->dx + B * r->dy);
          gg[1] += gs * (B * r->dx + C * r->dy);
        }
        for (int c = 0; c < 3; ++c) S[c] += c3[c] * w;
        SD += z * w;
      }
    }
  }
  free(list);
  return NULL;
}

static int cmp_depth_index(const void *pa, const void *pb, void *ctx) {
  const double *depth = (const double *)ctx;
  const int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
  if (depth[a] < depth[b]) return -1;
  if (depth[a] > depth[b]) return 1;
  return (a > b) - (a < b);
}

/* Visible Gaussians whose conservative box meets the crop, in (depth, index)
 * order.  Returns the count; *out is malloc'ed. */
static int64_t build_order(const orc_proj *pr, int64_t n, int32_t x0, int32_t y0, int32_t cw, int32_t ch,
                           int64_t **out) {
  int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!pr->visible[i]) continue;
    const double rb = pr->radius[i] + 1.0;
    const double mx = pr->mean2d[i], my = pr->mean2d[n + i];
    if (mx + rb < x0 || mx - rb > x0 + cw - 1 || my + rb < y0 || my - rb > y0 + ch - 1) continue;
    ord[m++] = i;
  }
  qsort_r(ord, (size_t)m, sizeof(int64_t), cmp_depth_index, (void *)pr->depth);
  *out = ord;
  return m;
}

static int clamp_threads(int nthreads, int rows) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > ORC_MAX_THREADS) nthreads = ORC_MAX_THREADS;
  if (nthreads > rows) nthreads = rows > 0 ? rows : 1;
  return nthreads;
}

static void run_threads(render_job *jb, void *(*fn)(void *)) {
  pthread_t th[ORC_MAX_THREADS];
  render_task tasks[ORC_MAX_THREADS];
  for (int t = 0; t < jb->nthreads; ++t) {
    tasks[t].job = jb;
    tasks[t].tid = t;
    pthread_create(&th[t], NULL, fn, &tasks[t]);
  }
  for (int t = 0; t < jb->nthreads; ++t) pthread_join(th[t], NULL);
}

int orc_render(const orc_cam *cam, const orc_proj *pr, int64_t n, int32_t x0, int32_t y0, int32_t cw, int32_t ch,
               double flag_rel, int nthreads, double *image, double *depth, double *alpha, double *final_t,
               int32_t *n_contrib, int32_t *n_support, int32_t *flags) {
  if (cw <= 0 || ch <= 0) return 0;
  render_job jb;
  memset(&jb, 0, sizeof(jb));
  jb.cam = cam; jb.pr = pr; jb.n = n;
  jb.x0 = x0; jb.y0 = y0; jb.cw = cw; jb.ch = ch; jb.flag_rel = flag_rel;
  jb.image = image; jb.depth = depth; jb.alpha = alpha; jb.final_t = final_t;
  jb.n_contrib = n_contrib; jb.n_support = n_support; jb.flags = flags;
  int64_t *ord;
  jb.n_order = build_order(pr, n, x0, y0, cw, ch, &ord);
  jb.order = ord;
  jb.nthreads = clamp_threads(nthreads, ch);
  jb.rows_per = (ch + jb.nthreads - 1) / jb.nthreads;
  run_threads(&jb, render_fwd_worker);
  free(ord);
  return 0;
}

/* g2d: [n][10] (dmx, dmy, dA, dB, dC, do, dr, dg, db, dz), accumulated. */
int orc_render_bwd(const orc_cam *cam, const orc_proj *pr, int64_t n, int32_t x0, int32_t y0, int32_t cw, int32_t ch,
                   int nthreads, const double *g_image, const double *g_depth, const double *g_alpha, double *g2d) {
  if (cw <= 0 || ch <= 0) return 0;
  render_job jb;
  memset(&jb, 0, sizeof(jb));
  jb.cam = cam; jb.pr = pr; jb.n = n;
  jb.x0 = x0; jb.y0 = y0; jb.cw = cw; jb.ch = ch;
  jb.g_image = g_image; jb.g_depth = g_depth; jb.g_alpha = g_alpha;
  int64_t *ord;
  jb.n_order = build_order(pr, n, x0, y0, cw, ch, &ord);
  jb.order = ord;
  jb.nthreads = clamp_threads(nthreads, ch);
  jb.rows_per = (ch + jb.nthreads - 1) / jb.nthreads;
  const size_t per = (size_t)(jb.n_order > 0 ? jb.n_order : 1) * 10;
  jb.g2d_threads = (double *)calloc(per * (size_t)jb.nthreads, sizeof(double));
  if (!jb.g2d_threads) {
    free(ord);
    return -1;
  }
  run_threads(&jb, render_bwd_worker);
  for (int t = 0; t < jb.nthreads; ++t) {
    const double *src = jb.g2d_threads + per * (size_t)t;
    for (int64_t k = 0; k < jb.n_order; ++k)
      for (int j = 0; j < 10; ++j) g2d[ord[k] * 10 + j] += src[k * 10 + j];
  }
  free(jb.g2d_threads);
  free(ord);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Backward of the projection for every visible Gaussian.                     */
/*   g2d  [n][10]  gradients of the per-Gaussian 2D quantities                */
/*   grads accumulate into d_means [3][n], d_log_scales [3][n], d_quats       */
/*   [4][n], d_opacity_logits [n], d_sh [(deg+1)^2][3][n];                    */
/*   d_R [9] and d_t [3] accumulate the camera pose gradient, d_twist [6]     */
/*   accumulates the left-perturbation twist (rho, phi) of this call.         */
/* ------------------------------------------------------------------------ */
void orc_project_bwd(const orc_cam *cam, const orc_gauss *g, const double *g2d, double *d_means, double *d_log_scales,
                     double *d_quats, double *d_opacity_logits, double *d_sh, double *d_R, double *d_t,
                     double *d_twist) {
  const int64_t n = g->n;
  const double *R = cam->R;
  const int nb = (g->sh_degree + 1) * (g->sh_degree + 1);
  double sumR[9] = {0}, sumt[3] = {0};
  for (int64_t i = 0; i < n; ++i) {
    gfwd f;
    project_one(cam, g, i, &f);
    if (!f.visible) continue;
    const double *gi = g2d + i * 10;
    double gmu[3] = {0, 0, 0};

    /* colour: SH coefficients, and the mean through the view direction */
    {
      double Y[16], dY[16][3];
      sh_eval(g->sh_degree, f.dhat, Y, dY);
      double gdh[3] = {0, 0, 0};
      for (int ch = 0; ch < 3; ++ch) {
        if (f.clamped & (1 << ch)) continue;
        const double gv = gi[6 + ch];
        for (int k = 0; k < nb; ++k) {
          d_sh[(k * 3 + ch) * n + i] += gv * Y[k];
          const double coef = g->sh[(k * 3 + ch) * n + i];
          for (int a = 0; a < 3; ++a) gdh[a] += gv * coef * dY[k][a];
        }
      }
      const double dd = gdh[0] * f.dhat[0] + gdh[1] * f.dhat[1] + gdh[2] * f.dhat[2];
      for (int a = 0; a < 3; ++a) gmu[a] += (gdh[a] - f.dhat[a] * dd) / f.dnorm;
    }

    /* opacity logit: o = sigmoid(logit) rho */
    d_opacity_logits[i] += gi[5] * f.rho * f.osig * (1.0 - f.osig);

    /* conic -> Sigma2 (full-matrix gradient, symmetric) */
    const double Q[4] = {f.A, f.B, f.B, f.C};
    const double Gq[4] = {gi[2], 0.5 * gi[3], 0.5 * gi[3], gi[4]};
    double QG[4], gS2[4];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) QG[2 * r + c] = Q[2 * r] * Gq[c] + Q[2 * r + 1] * Gq[2 + c];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) gS2[2 * r + c] = -(QG[2 * r] * Q[c] + QG[2 * r + 1] * Q[2 + c]);
    if (cam->mip_filter) {
      /* rho^2 = det0 / det with det0 = a0 c0 - b^2, det = (a0 + eps)(c0 + eps) - b^2:
         d rho = d(rho^2) / (2 rho), quotient rule; the off-diagonal b sits in two entries */
      const double g_rho = gi[5] * f.osig, D0 = f.det0, D = f.det, k = g_rho / (2.0 * f.rho * D * D);
      gS2[0] += k * (f.c0 * D - D0 * f.c);
      gS2[3] += k * (f.a0 * D - D0 * f.a);
      const double gb = k * (-2.0 * f.b * D + 2.0 * f.b * D0);
      gS2[1] += 0.5 * gb;
      gS2[2] += 0.5 * gb;
    }

    /* Sigma2 = J V J^T + eps I:  gV = J^T gS2 J,  gJ = 2 gS2 J V */
    double gV[9], gJ[6], JV[6];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s = 0.0;
        for (int r = 0; r < 2; ++r)
          for (int c = 0; c < 2; ++c) s += f.J[3 * r + a] * gS2[2 * r + c] * f.J[3 * c + b];
        gV[3 * a + b] = s;
      }
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c)
        JV[3 * r + c] = f.J[3 * r] * f.V[c] + f.J[3 * r + 1] * f.V[3 + c] + f.J[3 * r + 2] * f.V[6 + c];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) gJ[3 * r + c] = 2.0 * (gS2[2 * r] * JV[c] + gS2[2 * r + 1] * JV[3 + c]);

    /* V = R Sigma R^T:  gSigma = R^T gV R,  gR_cov = 2 gV R Sigma */
    double tmp[9], gSig[9], gRcov[9];
    mat3_mul_at(R, gV, tmp);
    mat3_mul(tmp, R, gSig);
    double RSig[9];
    mat3_mul(R, f.Sig, RSig);
    mat3_mul(gV, RSig, gRcov);
    for (int k = 0; k < 9; ++k) gRcov[k] *= 2.0;

    /* Sigma = M M^T with M = Rq diag(s) */
    double gM[9];
    mat3_mul(gSig, f.M, gM);
    for (int k = 0; k < 9; ++k) gM[k] *= 2.0;
    double gRq[9], gs[3] = {0, 0, 0};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        gRq[3 * r + c] = gM[3 * r + c] * f.s[c];
        gs[c] += gM[3 * r + c] * f.Rq[3 * r + c];
      }
    for (int c = 0; c < 3; ++c) d_log_scales[c * n + i] += gs[c] * f.s[c];
    double gqn[4];
    quat_to_rot_vjp(f.qn, gRq, gqn);
    const double qd = gqn[0] * f.qn[0] + gqn[1] * f.qn[1] + gqn[2] * f.qn[2] + gqn[3] * f.qn[3];
    for (int k = 0; k < 4; ++k) d_quats[k * n + i] += (gqn[k] - f.qn[k] * qd) / f.qnorm;

    /* perspective: mean2d, depth and J as functions of p */
    const double z = f.z, z2 = z * z, z3 = z2 * z;
    const double gmx = gi[0], gmy = gi[1], gz = gi[9];
    double gp[3];
    gp[0] = gmx * cam->fx / z;
    gp[1] = gmy * cam->fy / z;
    gp[2] = gz - gmx * cam->fx * f.p[0] / z2 - gmy * cam->fy * f.p[1] / z2;
    gp[2] += -gJ[0] * cam->fx / z2 - gJ[4] * cam->fy / z2;
    if (!f.clx) {
      gp[0] += gJ[2] * (-cam->fx / z2);
      gp[2] += gJ[2] * (2.0 * cam->fx * f.p[0] / z3);
    } else {
      gp[2] += gJ[2] * (-f.J[2] / z);
    }
    if (!f.cly) {
      gp[1] += gJ[5] * (-cam->fy / z2);
      gp[2] += gJ[5] * (2.0 * cam->fy * f.p[1] / z3);
    } else {
      gp[2] += gJ[5] * (-f.J[5] / z);
    }

    /* p = R mu + t */
    const double mu[3] = {g->means[i], g->means[n + i], g->means[2 * n + i]};
    for (int a = 0; a < 3; ++a) gmu[a] += R[a] * gp[0] + R[3 + a] * gp[1] + R[6 + a] * gp[2];
    for (int a = 0; a < 3; ++a) d_means[a * n + i] += gmu[a];
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) sumR[3 * r + c] += gp[r] * mu[c] + gRcov[3 * r + c];
      sumt[r] += gp[r];
    }
  }
  for (int k = 0; k < 9; ++k) d_R[k] += sumR[k];
  for (int k = 0; k < 3; ++k) d_t[k] += sumt[k];
  if (d_twist) {
    /* left perturbation T <- exp(xi^) T, xi = (rho, phi):
       d/drho = dL/dt, d/dphi from M = dL/dR R^T + dL/dt t^T */
    double Mm[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += sumR[3 * r + k] * R[3 * c + k];
        Mm[3 * r + c] = s + sumt[r] * cam->t[c];
      }
    for (int k = 0; k < 3; ++k) d_twist[k] += sumt[k];
    d_twist[3] += Mm[7] - Mm[5];
    d_twist[4] += Mm[2] - Mm[6];
    d_twist[5] += Mm[3] - Mm[1];
  }
}
