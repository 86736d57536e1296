/*
 * pabd_oracle.c -- plain, slow, FP64 CPU oracle of projective affine body
 * dynamics (Ye, He, Guo, Yang, Jiang, Wang: "Projective Affine Body Dynamics for
 * Multibody Systems").
 *
 * TEST INFRASTRUCTURE ONLY.  Used by tests/, by the package smoke check and by
 * the CPU-baseline leg of the benchmark.  The HIP library never links or calls
 * it, and it shares no code with the library.
 *
 * What it computes, one simulation step (Algorithm 1 of the paper):
 *   1. collision detection on q^n, producing contact bonds (reading of the
 *      unpublished contact model, see contact_* below);
 *   2. prediction (Algorithm 1, prediction loop): v* = v + h g,
 *      c* = c + h v*, Q* = Q + h/2 [w,0] Q (normalised), q^0 = s = (c*, R(Q*));
 *   3. K iterations of the global/local alternation (Sec. 4.2):
 *      global: the body-wise Jacobi update of the global solve (Sec. 4.2.1),
 *        q^{k+1/2} = H^{-1} (M s + h^2 sum phi^- J^T n + h^2 sum phi^+/d J^T y_j),
 *        with H = M + h^2 sum phi^+/d J^T J assembled DENSE (12x12) and solved
 *        by Cholesky -- not the sparse closed form of Sec. 4.3;
 *      local: A^{k+1} = rotation factor of the polar decomposition of
 *        A^{k+1/2} (Sec. 4.2.2), computed through a Jacobi SVD; c unchanged;
 *   4. velocity recovery (Sec. 4.4): v = (c^{n+1} - c^n)/h,
 *      [w]_x = (A^{n+1} - A^n)(A^n)^{-1}/h, averaged with minus its transpose.
 *
 * Parity pins live in tests/test_oracle_*.py.
 */
#include "pabd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------- */
/* small dense linear algebra, written out plainly                            */
/* ------------------------------------------------------------------------- */

static void m3_mul(const double *a, const double *b, double *out) {
  double t[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += a[3 * r + k] * b[3 * k + c];
      t[3 * r + c] = s;
    }
  memcpy(out, t, sizeof t);
}

static void m3_transpose(const double *a, double *out) {
  double t[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) t[3 * r + c] = a[3 * c + r];
  memcpy(out, t, sizeof t);
}

static void m3_vec(const double *a, const double *x, double *out) {
  double t[3];
  for (int r = 0; r < 3; ++r) t[r] = a[3 * r] * x[0] + a[3 * r + 1] * x[1] + a[3 * r + 2] * x[2];
  memcpy(out, t, sizeof t);
}

static void m3_tvec(const double *a, const double *x, double *out) { /* a^T x */
  double t[3];
  for (int c = 0; c < 3; ++c) t[c] = a[c] * x[0] + a[3 + c] * x[1] + a[6 + c] * x[2];
  memcpy(out, t, sizeof t);
}

static double m3_det(const double *a) {
  return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
         a[2] * (a[3] * a[7] - a[4] * a[6]);
}

/* explicit inverse through the adjugate */
static int m3_inverse(const double *a, double *out) {
  double det = m3_det(a);
  if (det == 0.0) return -1;
  double t[9];
  t[0] = (a[4] * a[8] - a[5] * a[7]) / det;
  t[1] = (a[2] * a[7] - a[1] * a[8]) / det;
  t[2] = (a[1] * a[5] - a[2] * a[4]) / det;
  t[3] = (a[5] * a[6] - a[3] * a[8]) / det;
  t[4] = (a[0] * a[8] - a[2] * a[6]) / det;
  t[5] = (a[2] * a[3] - a[0] * a[5]) / det;
  t[6] = (a[3] * a[7] - a[4] * a[6]) / det;
  t[7] = (a[1] * a[6] - a[0] * a[7]) / det;
  t[8] = (a[0] * a[4] - a[1] * a[3]) / det;
  memcpy(out, t, sizeof t);
  return 0;
}

static double v3_dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double v3_norm(const double *a) { return sqrt(v3_dot(a, a)); }
static void v3_cross(const double *a, const double *b, double *out) {
  double t[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  memcpy(out, t, sizeof t);
}

/* Cholesky factorisation of an SPD n x n matrix (lower factor in place) */
static int cholesky(double *a, int n) {
  for (int j = 0; j < n; ++j) {
    double s = a[j * n + j];
    for (int k = 0; k < j; ++k) s -= a[j * n + k] * a[j * n + k];
    if (!(s > 0.0)) return -1;
    double ljj = sqrt(s);
    a[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = a[i * n + j];
      for (int k = 0; k < j; ++k) t -= a[i * n + k] * a[j * n + k];
      a[i * n + j] = t / ljj;
    }
    for (int i = 0; i < j; ++i) a[i * n + j] = 0.0;
  }
  return 0;
}

static void cholesky_solve(const double *l, int n, const double *b, double *x) {
  double y[12];
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= l[i * n + k] * y[k];
    y[i] = s / l[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < n; ++k) s -= l[k * n + i] * x[k];
    x[i] = s / l[i * n + i];
  }
}

/* cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix:
 * s = V diag(lam) V^T, eigenvalues sorted in decreasing order */
static void sym3_eigen(const double *s_in, double *lam, double *V) {
  double a[9];
  memcpy(a, s_in, sizeof a);
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
    double diag = a[0] * a[0] + a[4] * a[4] + a[8] * a[8];
    if (off <= 1e-300 || off <= 1e-34 * diag) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        double apq = a[3 * p + q];
        if (apq == 0.0) continue;
        double theta = (a[3 * q + q] - a[3 * p + p]) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        /* a <- G^T a G with the Givens rotation G acting on (p, q) */
        for (int k = 0; k < 3; ++k) {
          double akp = a[3 * k + p], akq = a[3 * k + q];
          a[3 * k + p] = c * akp - s * akq;
          a[3 * k + q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          double apk = a[3 * p + k], aqk = a[3 * q + k];
          a[3 * p + k] = c * apk - s * aqk;
          a[3 * q + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          double vkp = V[3 * k + p], vkq = V[3 * k + q];
          V[3 * k + p] = c * vkp - s * vkq;
          V[3 * k + q] = s * vkp + c * vkq;
        }
      }
  }
  double l[3] = {a[0], a[4], a[8]};
  /* sort descending, permuting the columns of V */
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2 - i; ++j)
      if (l[j] < l[j + 1]) {
        double t = l[j];
        l[j] = l[j + 1];
        l[j + 1] = t;
        for (int k = 0; k < 3; ++k) {
          double u = V[3 * k + j];
          V[3 * k + j] = V[3 * k + j + 1];
          V[3 * k + j + 1] = u;
        }
      }
  memcpy(lam, l, sizeof l);
}

/* Nearest rotation to A: A = U S V^T (SVD), R = U diag(1, 1, det(U V^T)) V^T.
 * For det A > 0 this is the rotation factor of the polar decomposition A = R S
 * (Sec. 4.2.2, local solve); for det A <= 0 it is the closest proper rotation. */
void pabd_oracle_polar(const double *A, double *R) {
  double At[9], AtA[9], lam[3], V[9];
  m3_transpose(A, At);
  m3_mul(At, A, AtA);
  sym3_eigen(AtA, lam, V);
  double sig[3], U[9];
  for (int k = 0; k < 3; ++k) sig[k] = sqrt(lam[k] > 0.0 ? lam[k] : 0.0);
  /* columns of U from A v_k / sigma_k; the last from a cross product when the
   * matrix is (nearly) rank deficient */
  for (int k = 0; k < 3; ++k) {
    double vk[3] = {V[k], V[3 + k], V[6 + k]}, u[3];
    m3_vec(A, vk, u);
    double nu = v3_norm(u);
    if (k < 2 || sig[2] > 1e-12 * sig[0]) {
      if (nu > 0.0)
        for (int r = 0; r < 3; ++r) U[3 * r + k] = u[r] / nu;
      else
        for (int r = 0; r < 3; ++r) U[3 * r + k] = (r == k) ? 1.0 : 0.0;
    } else {
      double u0[3] = {U[0], U[3], U[6]}, u1[3] = {U[1], U[4], U[7]}, u2[3];
      v3_cross(u0, u1, u2);
      for (int r = 0; r < 3; ++r) U[3 * r + 2] = u2[r];
    }
  }
  double Vt[9], UVt[9];
  m3_transpose(V, Vt);
  m3_mul(U, Vt, UVt);
  double dsign = m3_det(UVt) < 0.0 ? -1.0 : 1.0;
  double D[9] = {1, 0, 0, 0, 1, 0, 0, 0, dsign}, UD[9];
  m3_mul(U, D, UD);
  m3_mul(UD, Vt, R);
}

/* ------------------------------------------------------------------------- */
/* quaternions, scalar last (x, y, z, w), Hamilton product                    */
/* ------------------------------------------------------------------------- */

static void quat_mul(const double *p, const double *q, double *out) {
  double t[4];
  t[0] = p[3] * q[0] + q[3] * p[0] + (p[1] * q[2] - p[2] * q[1]);
  t[1] = p[3] * q[1] + q[3] * p[1] + (p[2] * q[0] - p[0] * q[2]);
  t[2] = p[3] * q[2] + q[3] * p[2] + (p[0] * q[1] - p[1] * q[0]);
  t[3] = p[3] * q[3] - (p[0] * q[0] + p[1] * q[1] + p[2] * q[2]);
  memcpy(out, t, sizeof t);
}

/* Shoemake: rotation matrix of a unit quaternion */
static void quat_to_mat(const double *q, double *R) {
  double x = q[0], y = q[1], z = q[2], w = q[3];
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - z * w);
  R[2] = 2 * (x * z + y * w);
  R[3] = 2 * (x * y + z * w);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - x * w);
  R[6] = 2 * (x * z - y * w);
  R[7] = 2 * (y * z + x * w);
  R[8] = 1 - 2 * (x * x + y * y);
}

/* Shepperd's method: unit quaternion of a rotation matrix */
static void mat_to_quat(const double *R, double *q) {
  double tr = R[0] + R[4] + R[8];
  double cand[4] = {R[0], R[4], R[8], tr};
  int big = 3;
  for (int k = 0; k < 3; ++k)
    if (cand[k] > cand[big]) big = k;
  if (big == 3) {
    double s = 2.0 * sqrt(1.0 + tr);
    q[3] = 0.25 * s;
    q[0] = (R[7] - R[5]) / s;
    q[1] = (R[2] - R[6]) / s;
    q[2] = (R[3] - R[1]) / s;
  } else if (big == 0) {
    double s = 2.0 * sqrt(1.0 + R[0] - R[4] - R[8]);
    q[0] = 0.25 * s;
    q[3] = (R[7] - R[5]) / s;
    q[1] = (R[1] + R[3]) / s;
    q[2] = (R[2] + R[6]) / s;
  } else if (big == 1) {
    double s = 2.0 * sqrt(1.0 + R[4] - R[0] - R[8]);
    q[1] = 0.25 * s;
    q[3] = (R[2] - R[6]) / s;
    q[0] = (R[1] + R[3]) / s;
    q[2] = (R[5] + R[7]) / s;
  } else {
    double s = 2.0 * sqrt(1.0 + R[8] - R[0] - R[4]);
    q[2] = 0.25 * s;
    q[3] = (R[3] - R[1]) / s;
    q[0] = (R[2] + R[6]) / s;
    q[1] = (R[5] + R[7]) / s;
  }
}

/* ------------------------------------------------------------------------- */
/* affine body kinematics (Sec. 3, affine map y = A x + c = J q)              */
/* ------------------------------------------------------------------------- */

/* q = (c, a1, a2, a3) with A = [a1, a2, a3]^T (rows) */
static void q_from_cA(const double *c, const double *A, double *q) {
  memcpy(q, c, 3 * sizeof(double));
  memcpy(q + 3, A, 9 * sizeof(double));
}

/* J = [I3, I3 (x) x^T]: the 3 x 12 Jacobian, written out as a matrix
 * (Sec. 4.3, the matrix form of J) */
static void jacobian(const double *x, double *J) {
  memset(J, 0, 36 * sizeof(double));
  for (int r = 0; r < 3; ++r) {
    J[12 * r + r] = 1.0;
    for (int k = 0; k < 3; ++k) J[12 * r + 3 + 3 * r + k] = x[k];
  }
}

static void apply_J(const double *x, const double *q, double *y) {
  double J[36];
  jacobian(x, J);
  for (int r = 0; r < 3; ++r) {
    double s = 0.0;
    for (int c = 0; c < 12; ++c) s += J[12 * r + c] * q[c];
    y[r] = s;
  }
}

/* out += scale * J^T f */
static void add_JT(const double *x, const double *f, double scale, double *out) {
  double J[36];
  jacobian(x, J);
  for (int c = 0; c < 12; ++c) {
    double s = 0.0;
    for (int r = 0; r < 3; ++r) s += J[12 * r + c] * f[r];
    out[c] += scale * s;
  }
}

/* H += scale * J^T J */
static void add_JTJ(const double *x, double scale, double *H) {
  double J[36];
  jacobian(x, J);
  for (int a = 0; a < 12; ++a)
    for (int b = 0; b < 12; ++b) {
      double s = 0.0;
      for (int r = 0; r < 3; ++r) s += J[12 * r + a] * J[12 * r + b];
      H[12 * a + b] += scale * s;
    }
}

/* mass and affine moment of inertia Pi = int rho x x^T dV in the body's
 * principal material frame (Sec. 4.1.1, Theorem on the generalised mass) */
void pabd_oracle_body_mass(int32_t shape, const double *param, double density, double *m,
                           double *Pi0) {
  memset(Pi0, 0, 9 * sizeof(double));
  if (shape == ORACLE_SHAPE_BOX) {
    double sx = 2 * param[0], sy = 2 * param[1], sz = 2 * param[2];
    *m = density * sx * sy * sz;
    Pi0[0] = *m * sx * sx / 12.0;
    Pi0[4] = *m * sy * sy / 12.0;
    Pi0[8] = *m * sz * sz / 12.0;
  } else {
    double r = param[0];
    *m = density * 4.0 / 3.0 * M_PI * r * r * r;
    Pi0[0] = Pi0[4] = Pi0[8] = *m * r * r / 5.0;
  }
}

/* 12x12 generalised mass M_i = diag(m I, Pi, Pi, Pi) */
static void mass_matrix(double m, const double *Pi, double *M) {
  memset(M, 0, 144 * sizeof(double));
  for (int r = 0; r < 3; ++r) M[12 * r + r] = m;
  for (int blk = 0; blk < 3; ++blk)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) M[12 * (3 + 3 * blk + r) + 3 + 3 * blk + c] = Pi[3 * r + c];
}

/* ------------------------------------------------------------------------- */
/* scene                                                                      */
/* ------------------------------------------------------------------------- */

typedef struct {
  int32_t i, j, type;
  double xi[3], xj[3];
  double kappa, rest;
  double normal[3]; /* contacts: unit normal of j's surface, pointing to i */
  double mu;
  int32_t feature;
  double al_kappa, al_lambda; /* augmented bonds: kappa_j^k, lambda_j^k */
  int32_t order;              /* polynomial bonds: p */
  double axis[3];             /* slider bonds: unit axis u of the line (j's frame) */
} bond_t;

struct pabd_oracle {
  int32_t n;
  int32_t *shape;
  double *param, *mass, *Pi, *radius;
  uint8_t *flags;
  int32_t *group;
  double *c, *A, *v, *w; /* state q^n */
  int32_t n_static;
  bond_t *static_bonds;
  double *drive;
  double gravity[3], h, t0;
  int32_t iters, contact_enable;
  double mu, kscale, margin;
  int32_t n_planes;
  double *planes;
  double al_beta, al_alpha, al_gamma;
  int64_t steps_done;
  int32_t debug;
  /* per step */
  bond_t *bonds;
  int32_t n_bonds, cap_bonds, n_contacts;
  int32_t *inc_start, *inc_bond, *inc_side;
  double *rho;
  double *q_prev, *q_half;
  double *H; /* [N*144] dense, per step */
};

static void free_all(pabd_oracle *o) {
  if (!o) return;
  free(o->shape); free(o->param); free(o->mass); free(o->Pi); free(o->radius);
  free(o->flags); free(o->group); free(o->c); free(o->A); free(o->v); free(o->w);
  free(o->static_bonds); free(o->drive); free(o->planes); free(o->bonds);
  free(o->inc_start); free(o->inc_bond); free(o->inc_side); free(o->rho);
  free(o->q_prev); free(o->q_half); free(o->H);
  free(o);
}

void pabd_oracle_destroy(pabd_oracle *o) { free_all(o); }

static int pinned(const pabd_oracle *o, int b) { return (o->flags[b] & ORACLE_FLAG_PINNED) != 0; }

pabd_oracle *pabd_oracle_create(const pabd_oracle_desc *d) {
  if (!d || d->n_bodies < 0 || d->n_bonds < 0 || !(d->h > 0.0) || d->iters < 1) return NULL;
  int n = d->n_bodies;
  pabd_oracle *o = (pabd_oracle *)calloc(1, sizeof *o);
  if (!o) return NULL;
  o->n = n;
  size_t nn = (size_t)(n > 0 ? n : 1);
  o->shape = calloc(nn, sizeof(int32_t));
  o->param = calloc(nn * 3, sizeof(double));
  o->mass = calloc(nn, sizeof(double));
  o->Pi = calloc(nn * 9, sizeof(double));
  o->radius = calloc(nn, sizeof(double));
  o->flags = calloc(nn, 1);
  o->group = calloc(nn, sizeof(int32_t));
  o->c = calloc(nn * 3, sizeof(double));
  o->A = calloc(nn * 9, sizeof(double));
  o->v = calloc(nn * 3, sizeof(double));
  o->w = calloc(nn * 3, sizeof(double));
  o->inc_start = calloc(nn + 1, sizeof(int32_t));
  o->rho = calloc((size_t)d->iters, sizeof(double));
  o->q_prev = calloc(nn * 12, sizeof(double));
  o->q_half = calloc(nn * 12, sizeof(double));
  o->H = calloc(nn * 144, sizeof(double));
  for (int b = 0; b < n; ++b) {
    o->shape[b] = d->shape[b];
    memcpy(o->param + 3 * b, d->shape_param + 3 * b, 3 * sizeof(double));
    o->flags[b] = d->flags ? d->flags[b] : 0;
    o->group[b] = d->group ? d->group[b] : 0;
    memcpy(o->c + 3 * b, d->c0 + 3 * b, 3 * sizeof(double));
    memcpy(o->A + 9 * b, d->A0 + 9 * b, 9 * sizeof(double));
    if (d->v0) memcpy(o->v + 3 * b, d->v0 + 3 * b, 3 * sizeof(double));
    if (d->w0) memcpy(o->w + 3 * b, d->w0 + 3 * b, 3 * sizeof(double));
    if (d->shape[b] != ORACLE_SHAPE_BOX && d->shape[b] != ORACLE_SHAPE_SPHERE) goto bad;
    pabd_oracle_body_mass(d->shape[b], d->shape_param + 3 * b, d->density ? d->density[b] : 0.0,
                          o->mass + b, o->Pi + 9 * b);
    if (d->mass) o->mass[b] = d->mass[b];
    if (d->Pi0) {
      /* packed symmetric 00 01 02 11 12 22 into the full 3 x 3 matrix */
      const double *p6 = d->Pi0 + 6 * b;
      double full[9] = {p6[0], p6[1], p6[2], p6[1], p6[3], p6[4], p6[2], p6[4], p6[5]};
      memcpy(o->Pi + 9 * b, full, sizeof full);
    }
    if (!pinned(o, b)) {
      if (!(o->mass[b] > 0.0)) goto bad;
      /* Pi0 positive definite: its Cholesky factorisation exists */
      double L[9];
      memcpy(L, o->Pi + 9 * b, sizeof L);
      if (cholesky(L, 3) != 0) goto bad;
    }
    {
      /* A0 must be a rotation: |A0^T A0 - I|_F <= 1e-6 and det A0 > 0 */
      const double *A = d->A0 + 9 * b;
      double At[9], AtA[9], e2 = 0.0;
      m3_transpose(A, At);
      m3_mul(At, A, AtA);
      for (int k = 0; k < 9; ++k) {
        double g = AtA[k] - (k % 4 == 0 ? 1.0 : 0.0);
        e2 += g * g;
      }
      if (!(e2 <= 1e-12) || !(m3_det(A) > 0.0)) goto bad;
    }
    o->radius[b] = d->shape[b] == ORACLE_SHAPE_BOX ? v3_norm(d->shape_param + 3 * b)
                                                     : d->shape_param[3 * b];
    if (pinned(o, b)) {
      memset(o->v + 3 * b, 0, 3 * sizeof(double));
      memset(o->w + 3 * b, 0, 3 * sizeof(double));
    }
  }
  o->n_static = d->n_bonds;
  o->static_bonds = calloc((size_t)(d->n_bonds > 0 ? d->n_bonds : 1), sizeof(bond_t));
  o->drive = calloc((size_t)(d->n_bonds > 0 ? d->n_bonds : 1) * 13, sizeof(double));
  for (int e = 0; e < d->n_bonds; ++e) {
    bond_t *bd = &o->static_bonds[e];
    bd->i = d->bond_i[e];
    bd->j = d->bond_j[e];
    bd->type = d->bond_type ? d->bond_type[e] : ORACLE_BOND_QUADRATIC;
    if (bd->i < 0 || bd->i >= n || bd->j < -1 || bd->j >= n || bd->i == bd->j) goto bad;
    if (bd->type != ORACLE_BOND_QUADRATIC && bd->type != ORACLE_BOND_DRIVEN &&
        bd->type != ORACLE_BOND_AUGMENTED && bd->type != ORACLE_BOND_POLYNOMIAL &&
        bd->type != ORACLE_BOND_SLIDER)
      goto bad;
    if (bd->type == ORACLE_BOND_POLYNOMIAL) {
      bd->order = d->order ? d->order[e] : 0;
      if (bd->order < 2 || bd->order % 2 != 0 || bd->order > 12) goto bad;
    }
    memcpy(bd->xi, d->x_i + 3 * e, 3 * sizeof(double));
    memcpy(bd->xj, d->x_j + 3 * e, 3 * sizeof(double));
    bd->kappa = d->kappa[e];
    bd->rest = d->rest_len ? d->rest_len[e] : 0.0;
    if (!(bd->kappa > 0.0) || bd->rest < 0.0) goto bad;
    /* an augmented bond needs l > 0: with l = 0 the elongation d >= 0 never
     * changes sign and the multiplier could only grow */
    if (bd->type == ORACLE_BOND_AUGMENTED && !(bd->rest > 0.0)) goto bad;
    /* first step: kappa^0 = kappa_start, lambda = 0 */
    bd->al_kappa = bd->kappa;
    bd->al_lambda = 0.0;
    if (bd->type == ORACLE_BOND_DRIVEN) {
      if (!d->drive) goto bad;
      memcpy(o->drive + 13 * e, d->drive + 13 * e, 13 * sizeof(double));
    }
    if (bd->type == ORACLE_BOND_SLIDER) {
      if (!d->drive || bd->rest != 0.0) goto bad;
      const double un = v3_norm(d->drive + 13 * e);
      if (!(un > 0.0) || !isfinite(un)) goto bad;
      for (int k = 0; k < 3; ++k) bd->axis[k] = d->drive[13 * e + k] / un;
    }
  }
  memcpy(o->gravity, d->gravity, sizeof o->gravity);
  o->h = d->h;
  o->t0 = d->t0;
  o->iters = d->iters;
  o->contact_enable = d->contact_enable;
  o->mu = d->mu;
  o->kscale = d->contact_kappa_scale;
  o->margin = d->contact_margin;
  o->al_beta = d->al_beta;
  o->al_alpha = d->al_alpha;
  o->al_gamma = d->al_gamma;
  o->n_planes = d->n_planes;
  o->planes = calloc((size_t)(d->n_planes > 0 ? d->n_planes : 1) * 4, sizeof(double));
  if (d->n_planes > 0) memcpy(o->planes, d->planes, (size_t)d->n_planes * 4 * sizeof(double));
  return o;
bad:
  free_all(o);
  return NULL;
}

void pabd_oracle_set_debug(pabd_oracle *o, int32_t flags) { o->debug = flags; }

void pabd_oracle_read_state(const pabd_oracle *o, double *c, double *A, double *v, double *w) {
  size_t n = (size_t)o->n;
  if (c) memcpy(c, o->c, n * 3 * sizeof(double));
  if (A) memcpy(A, o->A, n * 9 * sizeof(double));
  if (v) memcpy(v, o->v, n * 3 * sizeof(double));
  if (w) memcpy(w, o->w, n * 3 * sizeof(double));
}

int pabd_oracle_residuals(const pabd_oracle *o, double *rho, int32_t cap) {
  for (int k = 0; k < o->iters && k < cap; ++k) rho[k] = o->rho[k];
  return o->iters;
}

void pabd_oracle_last_iterates(const pabd_oracle *o, double *q_prev, double *q_half) {
  if (q_prev) memcpy(q_prev, o->q_prev, (size_t)o->n * 12 * sizeof(double));
  if (q_half) memcpy(q_half, o->q_half, (size_t)o->n * 12 * sizeof(double));
}

void pabd_oracle_dense_H(const pabd_oracle *o, int32_t body, double *H) {
  memcpy(H, o->H + (size_t)body * 144, 144 * sizeof(double));
}

void pabd_oracle_bond_state(const pabd_oracle *o, double *kappa, double *lambda) {
  for (int e = 0; e < o->n_static; ++e) {
    const bond_t *b = &o->static_bonds[e];
    const int al = b->type == ORACLE_BOND_AUGMENTED;
    if (kappa) kappa[e] = al ? b->al_kappa : b->kappa;
    if (lambda) lambda[e] = al ? b->al_lambda : 0.0;
  }
}

int pabd_oracle_contacts(const pabd_oracle *o, int32_t cap, int32_t *ci, int32_t *cj,
                         int32_t *feature, double *xi, double *xj, double *normal,
                         double *kappa) {
  int k = 0;
  for (int e = o->n_static; e < o->n_bonds; ++e, ++k) {
    if (k >= cap) continue;
    const bond_t *b = &o->bonds[e];
    if (ci) ci[k] = b->i;
    if (cj) cj[k] = b->j;
    if (feature) feature[k] = b->feature;
    if (xi) memcpy(xi + 3 * k, b->xi, 3 * sizeof(double));
    if (xj) memcpy(xj + 3 * k, b->xj, 3 * sizeof(double));
    if (normal) memcpy(normal + 3 * k, b->normal, 3 * sizeof(double));
    if (kappa) kappa[k] = b->kappa;
  }
  return o->n_contacts;
}

/* ------------------------------------------------------------------------- */
/* bonds of the current step                                                  */
/* ------------------------------------------------------------------------- */

static void push_bond(pabd_oracle *o, const bond_t *b) {
  if (o->n_bonds == o->cap_bonds) {
    o->cap_bonds = o->cap_bonds ? 2 * o->cap_bonds : 64;
    o->bonds = realloc(o->bonds, (size_t)o->cap_bonds * sizeof(bond_t));
  }
  o->bonds[o->n_bonds++] = *b;
}

/* Rodrigues rotation of vector p about unit axis u by angle th */
static void rotate_about(const double *u, double th, const double *p, double *out) {
  double cu[3], c = cos(th), s = sin(th), ud = v3_dot(u, p);
  v3_cross(u, p, cu);
  for (int k = 0; k < 3; ++k) out[k] = p[k] * c + cu[k] * s + u[k] * ud * (1.0 - c);
}

/* Driven joint target (a reading; the paper drives hinge angles with a periodic
 * function, Sec. 5.3.3): the j-side anchor is base rotated about the axis through
 * pivot by theta(t) = theta0 + amp sin(2 pi f t + phase). */
static void driven_anchor(const double *dr, double t, double *xj) {
  double th = dr[9] + dr[10] * sin(2.0 * M_PI * dr[11] * t + dr[12]);
  double rel[3] = {dr[6] - dr[3], dr[7] - dr[4], dr[8] - dr[5]}, rot[3];
  rotate_about(dr, th, rel, rot);
  for (int k = 0; k < 3; ++k) xj[k] = dr[3 + k] + rot[k];
}

/* ---- collision detection: reading of the contact bond ---------------------
 * The paper states that contact and friction are modelled as bonds (Sec. 4.2)
 * with Coulomb friction after Andrews et al. (Sec. 5) but gives the energies only
 * in its supplement.  Reading used here: at detection on q^n, each contact is a
 * bond between a point x_i of body i (box vertex or sphere surface point) and the
 * closest point x_j on the surface of j (material frame of j, or world
 * coordinates for a plane), with a fixed unit normal n (outward from j, towards
 * i) and stiffness kappa_c = scale * m_max / h^2.  The stick force on i is
 * f = kappa_c (y_j - y_i); it acts only while n.(y_i - y_j) < 0, and its
 * tangential part is clamped to mu times its normal part. */

/* speculative detection margin of a body: its surface can move by about
 * h (|v| + |w| R) within the step; a sphere's distance to anything does not
 * change when it spins about its centre, so spheres omit the |w| R term */
static double body_margin(const pabd_oracle *o, int b) {
  double spin = o->shape[b] == ORACLE_SHAPE_BOX ? v3_norm(o->w + 3 * b) * o->radius[b] : 0.0;
  return o->margin + o->h * (v3_norm(o->v + 3 * b) + spin);
}

static double contact_kappa(const pabd_oracle *o, int i, int j) {
  /* kappa_c = scale * m / h^2 with m the larger free mass of the pair (reading) */
  double m = 0.0;
  if (i >= 0 && !pinned(o, i)) m = o->mass[i];
  if (j >= 0 && !pinned(o, j) && o->mass[j] > m) m = o->mass[j];
  return o->kscale * m / (o->h * o->h);
}

static void box_vertex(int k, const double *he, double *x) {
  x[0] = (k & 1) ? he[0] : -he[0];
  x[1] = (k & 2) ? he[1] : -he[1];
  x[2] = (k & 4) ? he[2] : -he[2];
}

static void add_contact(pabd_oracle *o, int i, int j, int feature, const double *xi,
                        const double *xj, const double *n) {
  bond_t b;
  memset(&b, 0, sizeof b);
  b.i = i;
  b.j = j;
  b.type = ORACLE_BOND_CONTACT;
  b.feature = feature;
  memcpy(b.xi, xi, sizeof b.xi);
  memcpy(b.xj, xj, sizeof b.xj);
  memcpy(b.normal, n, sizeof b.normal);
  b.kappa = contact_kappa(o, i, j);
  b.mu = o->mu;
  push_bond(o, &b);
  o->n_contacts++;
}

static int may_collide(const pabd_oracle *o, int i, int j) {
  if ((o->flags[i] | o->flags[j]) & ORACLE_FLAG_NO_CONTACT) return 0;
  if (pinned(o, i) && pinned(o, j)) return 0;
  if (o->group[i] != 0 && o->group[i] == o->group[j]) return 0;
  return 1;
}

/* sphere s against box b (sphere is the i side) */
static void sphere_box(pabd_oracle *o, int s, int b, double pm) {
  const double *he = o->param + 3 * b, *Ab = o->A + 9 * b, *cb = o->c + 3 * b;
  const double *cs = o->c + 3 * s;
  double r = o->param[3 * s];
  double rel[3] = {cs[0] - cb[0], cs[1] - cb[1], cs[2] - cb[2]}, pl[3], q[3], nl[3];
  m3_tvec(Ab, rel, pl);
  int inside = 1;
  for (int k = 0; k < 3; ++k) {
    q[k] = pl[k] < -he[k] ? -he[k] : (pl[k] > he[k] ? he[k] : pl[k]);
    if (q[k] != pl[k]) inside = 0;
  }
  double gap;
  if (inside) {
    int ks = 0;
    double best = he[0] - fabs(pl[0]);
    for (int k = 1; k < 3; ++k)
      if (he[k] - fabs(pl[k]) < best) best = he[k] - fabs(pl[k]), ks = k;
    double sgn = pl[ks] >= 0.0 ? 1.0 : -1.0;
    q[ks] = sgn * he[ks];
    nl[0] = nl[1] = nl[2] = 0.0;
    nl[ks] = sgn;
    gap = -best - r;
  } else {
    double dl[3] = {pl[0] - q[0], pl[1] - q[1], pl[2] - q[2]};
    double dist = v3_norm(dl);
    if (dist == 0.0) return;
    for (int k = 0; k < 3; ++k) nl[k] = dl[k] / dist;
    gap = dist - r;
  }
  if (!(gap < pm)) return;
  double nw[3], pw[3], xi[3];
  m3_vec(Ab, nl, nw);
  for (int k = 0; k < 3; ++k) pw[k] = -r * nw[k];
  m3_tvec(o->A + 9 * s, pw, xi);
  add_contact(o, s, b, 8, xi, q, nw);
}

/* half-length of the projection of box b onto the unit axis u */
static double box_radius_along(const pabd_oracle *o, int b, const double *u) {
  const double *A = o->A + 9 * b, *he = o->param + 3 * b;
  double r = 0.0;
  for (int k = 0; k < 3; ++k) {
    double ek[3] = {A[k], A[3 + k], A[6 + k]}; /* k-th material axis in world */
    r += he[k] * fabs(v3_dot(u, ek));
  }
  return r;
}

/* box i against box j, vertex-face only.  The reference face is the face axis
 * (3 of i, then 3 of j) along which the two boxes overlap least; every vertex of
 * the other (incident) box that lies within the margin of that face, inside its
 * lateral extent, becomes a contact with the face's outward normal. */
static void box_box(pabd_oracle *o, int i, int j, double pm) {
  double dc[3] = {o->c[3 * j] - o->c[3 * i], o->c[3 * j + 1] - o->c[3 * i + 1],
                  o->c[3 * j + 2] - o->c[3 * i + 2]};
  int best_axis = -1;
  double best = 0.0;
  for (int ax = 0; ax < 6; ++ax) {
    int owner = ax < 3 ? i : j, k = ax % 3;
    const double *A = o->A + 9 * owner;
    double u[3] = {A[k], A[3 + k], A[6 + k]};
    double overlap = box_radius_along(o, i, u) + box_radius_along(o, j, u) - fabs(v3_dot(u, dc));
    if (overlap < -pm) return; /* separated along a face axis by more than the margin */
    if (best_axis < 0 || overlap < best) best = overlap, best_axis = ax;
  }
  int ref = best_axis < 3 ? i : j, inc = best_axis < 3 ? j : i, k = best_axis % 3;
  const double *Ar = o->A + 9 * ref, *cr = o->c + 3 * ref, *her = o->param + 3 * ref;
  const double *Ai = o->A + 9 * inc, *ci = o->c + 3 * inc, *hei = o->param + 3 * inc;
  double axis[3] = {Ar[k], Ar[3 + k], Ar[6 + k]};
  double towards[3] = {ci[0] - cr[0], ci[1] - cr[1], ci[2] - cr[2]};
  double sgn = v3_dot(axis, towards) >= 0.0 ? 1.0 : -1.0;
  double nw[3] = {sgn * axis[0], sgn * axis[1], sgn * axis[2]};
  for (int vtx = 0; vtx < 8; ++vtx) {
    double xv[3], p[3], rel[3], pl[3], xs[3];
    box_vertex(vtx, hei, xv);
    m3_vec(Ai, xv, p);
    for (int r = 0; r < 3; ++r) rel[r] = p[r] + ci[r] - cr[r];
    m3_tvec(Ar, rel, pl); /* rotation: inverse = transpose */
    double gap = sgn * pl[k] - her[k];
    if (!(gap < pm) || gap < -2.0 * her[k]) continue;
    int lateral = 1;
    for (int m = 0; m < 3; ++m)
      if (m != k && fabs(pl[m]) > her[m] + pm) lateral = 0;
    if (!lateral) continue;
    for (int m = 0; m < 3; ++m) xs[m] = pl[m] < -her[m] ? -her[m] : (pl[m] > her[m] ? her[m] : pl[m]);
    xs[k] = sgn * her[k];
    add_contact(o, inc, ref, vtx, xv, xs, nw);
  }
}

static void detect_pair(pabd_oracle *o, int i, int j) {
  double pm = body_margin(o, i) + body_margin(o, j);
  double dc[3] = {o->c[3 * j] - o->c[3 * i], o->c[3 * j + 1] - o->c[3 * i + 1],
                  o->c[3 * j + 2] - o->c[3 * i + 2]};
  double dist = v3_norm(dc);
  if (dist >= o->radius[i] + o->radius[j] + pm) return;
  int si = o->shape[i], sj = o->shape[j];
  if (si == ORACLE_SHAPE_BOX && sj == ORACLE_SHAPE_BOX) {
    box_box(o, i, j, pm);
  } else if (si == ORACLE_SHAPE_SPHERE && sj == ORACLE_SHAPE_SPHERE) {
    double gap = dist - o->param[3 * i] - o->param[3 * j];
    if (!(gap < pm) || dist == 0.0) return;
    double n[3] = {-dc[0] / dist, -dc[1] / dist, -dc[2] / dist}; /* from j towards i */
    double pi_[3], pj[3], xi[3], xj[3];
    for (int k = 0; k < 3; ++k) pi_[k] = -o->param[3 * i] * n[k], pj[k] = o->param[3 * j] * n[k];
    m3_tvec(o->A + 9 * i, pi_, xi);
    m3_tvec(o->A + 9 * j, pj, xj);
    add_contact(o, i, j, 8, xi, xj, n);
  } else if (si == ORACLE_SHAPE_SPHERE) {
    sphere_box(o, i, j, pm);
  } else {
    sphere_box(o, j, i, pm);
  }
}

static void detect_planes(pabd_oracle *o, int i) {
  double pm = body_margin(o, i);
  for (int p = 0; p < o->n_planes; ++p) {
    const double *n = o->planes + 4 * p;
    double off = n[3];
    if (o->shape[i] == ORACLE_SHAPE_BOX) {
      for (int k = 0; k < 8; ++k) {
        double x[3], y[3];
        box_vertex(k, o->param + 3 * i, x);
        m3_vec(o->A + 9 * i, x, y);
        for (int r = 0; r < 3; ++r) y[r] += o->c[3 * i + r];
        double gap = v3_dot(n, y) - off;
        if (gap < pm) {
          double xw[3] = {y[0] - gap * n[0], y[1] - gap * n[1], y[2] - gap * n[2]};
          add_contact(o, i, -1, 16 * p + k, x, xw, n);
        }
      }
    } else {
      double r = o->param[3 * i];
      double gap = v3_dot(n, o->c + 3 * i) - r - off;
      if (gap < pm) {
        double pw[3] = {-r * n[0], -r * n[1], -r * n[2]}, x[3];
        m3_tvec(o->A + 9 * i, pw, x);
        double xw[3];
        for (int k = 0; k < 3; ++k) xw[k] = o->c[3 * i + k] - (r + gap) * n[k];
        add_contact(o, i, -1, 16 * p + 8, x, xw, n);
      }
    }
  }
}

/* brute force over all pairs: obviously complete */
static void collision_detection(pabd_oracle *o) {
  for (int i = 0; i < o->n; ++i) {
    if (!pinned(o, i) && !(o->flags[i] & ORACLE_FLAG_NO_CONTACT)) detect_planes(o, i);
    for (int j = i + 1; j < o->n; ++j)
      if (may_collide(o, i, j)) detect_pair(o, i, j);
  }
}

static void build_bonds(pabd_oracle *o, double t) {
  o->n_bonds = 0;
  o->n_contacts = 0;
  for (int e = 0; e < o->n_static; ++e) {
    bond_t b = o->static_bonds[e];
    if (b.type == ORACLE_BOND_DRIVEN) driven_anchor(o->drive + 13 * e, t, b.xj);
    push_bond(o, &b);
  }
  if (o->contact_enable) collision_detection(o);
  /* per-body incidence lists, in bond order */
  int n = o->n;
  memset(o->inc_start, 0, (size_t)(n + 1) * sizeof(int32_t));
  for (int e = 0; e < o->n_bonds; ++e) {
    o->inc_start[o->bonds[e].i + 1]++;
    if (o->bonds[e].j >= 0) o->inc_start[o->bonds[e].j + 1]++;
  }
  for (int b = 0; b < n; ++b) o->inc_start[b + 1] += o->inc_start[b];
  int total = o->inc_start[n];
  free(o->inc_bond);
  free(o->inc_side);
  o->inc_bond = calloc((size_t)(total > 0 ? total : 1), sizeof(int32_t));
  o->inc_side = calloc((size_t)(total > 0 ? total : 1), sizeof(int32_t));
  int32_t *fill = calloc((size_t)n + 1, sizeof(int32_t));
  for (int e = 0; e < o->n_bonds; ++e) {
    int i = o->bonds[e].i, j = o->bonds[e].j;
    int pi_ = o->inc_start[i] + fill[i]++;
    o->inc_bond[pi_] = e;
    o->inc_side[pi_] = 0;
    if (j >= 0) {
      int pj = o->inc_start[j] + fill[j]++;
      o->inc_bond[pj] = e;
      o->inc_side[pj] = 1;
    }
  }
  free(fill);
}

int pabd_oracle_detect(pabd_oracle *o) {
  build_bonds(o, o->t0 + (double)(o->steps_done + 1) * o->h);
  return o->n_contacts;
}

/* the contacts of one body on the current state, by the same rule: its plane
 * contacts and every pair (lower index first) that contains it, against all
 * other bodies -- O(N), for sampled checks of large scenes */
int pabd_oracle_detect_body(pabd_oracle *o, int32_t body) {
  if (body < 0 || body >= o->n) return -1;
  o->n_bonds = 0;
  o->n_contacts = 0;
  for (int e = 0; e < o->n_static; ++e) push_bond(o, &o->static_bonds[e]);
  if (!o->contact_enable) return 0;
  const int i = body;
  if (!pinned(o, i) && !(o->flags[i] & ORACLE_FLAG_NO_CONTACT)) detect_planes(o, i);
  for (int j = 0; j < o->n; ++j) {
    if (j == i) continue;
    const int a = i < j ? i : j, b = i < j ? j : i;
    if (may_collide(o, a, b)) detect_pair(o, a, b);
  }
  return o->n_contacts;
}

/* world point of a bond end at iterate q (all bodies, 12 per body) */
static void end_point(const double *q, int body, const double *x, double *y) {
  if (body < 0) {
    memcpy(y, x, 3 * sizeof(double));
    return;
  }
  apply_J(x, q + 12 * body, y);
}

/* slider bond at iterate q: the material point xf = x_j + t u of j (world
 * coordinates if j = -1) whose world image yf is the foot of the perpendicular
 * from y_i onto the line, t = (y_i - y_j(x_j)).g / g.g with g the line's world
 * direction (A_j u, or u) */
static void slider_foot(const double *q, const bond_t *b, double *xf, double *yf) {
  double yi[3], y0[3], g[3];
  end_point(q, b->i, b->xi, yi);
  end_point(q, b->j, b->xj, y0);
  if (b->j < 0)
    memcpy(g, b->axis, sizeof g);
  else
    m3_vec(q + 12 * b->j + 3, b->axis, g);
  const double dv[3] = {yi[0] - y0[0], yi[1] - y0[1], yi[2] - y0[2]};
  const double t = v3_dot(dv, g) / v3_dot(g, g);
  for (int k = 0; k < 3; ++k) xf[k] = b->xj[k] + t * b->axis[k];
  end_point(q, b->j, xf, yf);
}

/* contact force on the i side at iterate q (reading above) */
static void contact_force(const bond_t *b, const double *yi, const double *yj, double *f) {
  double d[3] = {yj[0] - yi[0], yj[1] - yi[1], yj[2] - yi[2]};
  double gap = -v3_dot(b->normal, d);
  if (!(gap < 0.0)) {
    f[0] = f[1] = f[2] = 0.0;
    return;
  }
  double fn = b->kappa * (-gap);
  double ft[3];
  for (int k = 0; k < 3; ++k) ft[k] = b->kappa * d[k] - fn * b->normal[k];
  double ftn = v3_norm(ft);
  if (ftn > b->mu * fn) {
    double s = b->mu * fn / ftn;
    for (int k = 0; k < 3; ++k) ft[k] *= s;
  }
  for (int k = 0; k < 3; ++k) f[k] = fn * b->normal[k] + ft[k];
}

/* Polynomial bond Psi = kappa / p (d - l)^p (p even): phi = kappa (d - l)^{p-1} =
 * kappa sum_k C(p-1, k) d^k (-l)^{p-1-k}.  For d, l >= 0 the terms with p-1-k even
 * are >= 0 and the others <= 0, which gives the split of Sec. 4.2.1:
 * phi^+ = kappa sum_{p-1-k even} C(p-1, k) d^k l^{p-1-k} (implicit) and
 * phi^- = -kappa sum_{p-1-k odd} C(p-1, k) d^k l^{p-1-k} (explicit).  p - 1 is
 * odd, so the k = 0 term is in phi^- and phi^+ / d is finite at d = 0. */
void pabd_oracle_poly_split(double kappa, int32_t p, double l, double d, double *wplus,
                            double *phim) {
  double binom = 1.0; /* C(p-1, k) */
  double wp = 0.0, pm = 0.0;
  for (int k = 0; k <= p - 1; ++k) {
    if (k > 0) binom = binom * (double)(p - k) / (double)k;
    const double lp = pow(l, (double)(p - 1 - k));
    if ((p - 1 - k) % 2 == 0) {
      wp += binom * (k >= 1 ? pow(d, (double)(k - 1)) : 0.0) * lp; /* term / d */
    } else {
      pm -= binom * pow(d, (double)k) * lp;
    }
  }
  *wplus = kappa * wp;
  *phim = kappa * pm;
}

/* M-weighted squared norm q^T M q of one body */
static double m_norm2(double m, const double *Pi, const double *q) {
  double s = m * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
  for (int blk = 0; blk < 3; ++blk) {
    double t[3];
    m3_vec(Pi, q + 3 + 3 * blk, t);
    s += v3_dot(q + 3 + 3 * blk, t);
  }
  return s;
}

static int one_step(pabd_oracle *o) {
  const int n = o->n;
  const double h = o->h, h2 = h * h;
  const double t = o->t0 + (double)(o->steps_done + 1) * h;

  /* augmented bonds, warm start (Sec. 5.2.2): kappa^0 = max(gamma kappa^n,
   * kappa_start), lambda^0 = alpha gamma lambda^n (on the first step this keeps
   * kappa_start and 0) */
  for (int e = 0; e < o->n_static; ++e) {
    bond_t *b = &o->static_bonds[e];
    if (b->type != ORACLE_BOND_AUGMENTED) continue;
    b->al_kappa = fmax(o->al_gamma * b->al_kappa, b->kappa);
    b->al_lambda = o->al_alpha * o->al_gamma * b->al_lambda;
  }

  /* Algorithm 1: collision detection */
  build_bonds(o, t);

  /* Algorithm 1: prediction loop */
  double *s = calloc((size_t)(n > 0 ? n : 1) * 12, sizeof(double));
  double *qk = calloc((size_t)(n > 0 ? n : 1) * 12, sizeof(double));
  double *qnext = calloc((size_t)(n > 0 ? n : 1) * 12, sizeof(double));
  for (int b = 0; b < n; ++b) {
    if (pinned(o, b)) {
      q_from_cA(o->c + 3 * b, o->A + 9 * b, s + 12 * b);
      continue;
    }
    double vs[3], cs[3];
    for (int k = 0; k < 3; ++k) vs[k] = o->v[3 * b + k] + h * o->gravity[k]; /* f_ext / m = g */
    for (int k = 0; k < 3; ++k) cs[k] = o->c[3 * b + k] + h * vs[k];
    double Q[4], wq[4] = {o->w[3 * b], o->w[3 * b + 1], o->w[3 * b + 2], 0.0}, dQ[4], Qs[4];
    mat_to_quat(o->A + 9 * b, Q);
    quat_mul(wq, Q, dQ);
    for (int k = 0; k < 4; ++k) Qs[k] = Q[k] + 0.5 * h * dQ[k];
    double qnorm = sqrt(Qs[0] * Qs[0] + Qs[1] * Qs[1] + Qs[2] * Qs[2] + Qs[3] * Qs[3]);
    for (int k = 0; k < 4; ++k) Qs[k] /= qnorm;
    double As[9];
    quat_to_mat(Qs, As);
    q_from_cA(cs, As, s + 12 * b);
  }
  memcpy(qk, s, (size_t)n * 12 * sizeof(double));

  /* Algorithm 1: K iterations of global solve + local solve.
   * H_i^k = M_i + h^2 sum w J^T J (Sec. 4.2.1, block matrix H) with
   * w = phi^+(d^k)/d^k: kappa for quadratic bonds (constant), and for a contact
   * bond kappa_c while it penetrates at iterate k, 0 otherwise (reading).  H is
   * assembled dense and solved by Cholesky every iteration. */
  int status = 0;
  double *al_C = calloc((size_t)(o->n_static > 0 ? o->n_static : 1), sizeof(double));
  for (int k = 0; k < o->iters && status == 0; ++k) {
    double num = 0.0, den = 0.0;
    /* augmented bonds: elongation C^k = d - l at the iterate q^k the forces of
     * this iteration use (reading) */
    for (int e = 0; e < o->n_static; ++e) {
      const bond_t *bd = &o->bonds[e];
      if (bd->type != ORACLE_BOND_AUGMENTED) continue;
      double yi[3], yj[3];
      end_point(qk, bd->i, bd->xi, yi);
      end_point(qk, bd->j, bd->xj, yj);
      double dv[3] = {yj[0] - yi[0], yj[1] - yi[1], yj[2] - yi[2]};
      al_C[e] = v3_norm(dv) - bd->rest;
    }
    for (int b = 0; b < n; ++b) {
      if (pinned(o, b)) {
        memcpy(qnext + 12 * b, qk + 12 * b, 12 * sizeof(double));
        continue;
      }
      double *H = o->H + 144 * (size_t)b;
      double r[12];
      mass_matrix(o->mass[b], o->Pi + 9 * b, H);
      for (int a = 0; a < 12; ++a) {
        double acc = 0.0;
        for (int c = 0; c < 12; ++c) acc += H[12 * a + c] * s[12 * b + c];
        r[a] = acc; /* M_i s_i */
      }
      for (int p = o->inc_start[b]; p < o->inc_start[b + 1]; ++p) {
        const bond_t *bd = &o->bonds[o->inc_bond[p]];
        int side = o->inc_side[p];
        int self = side ? bd->j : bd->i, other = side ? bd->i : bd->j;
        const double *xs = side ? bd->xj : bd->xi, *xo = side ? bd->xi : bd->xj;
        double ys[3], yo[3];
        end_point(qk, self, xs, ys);
        end_point(qk, other, xo, yo);
        if (bd->type == ORACLE_BOND_CONTACT) {
          double yi[3], yj[3], f[3], fe[3];
          memcpy(yi, side ? yo : ys, sizeof yi);
          memcpy(yj, side ? ys : yo, sizeof yj);
          double gap = bd->normal[0] * (yi[0] - yj[0]) + bd->normal[1] * (yi[1] - yj[1]) +
                       bd->normal[2] * (yi[2] - yj[2]);
          if (!(gap < 0.0)) continue; /* separated at iterate k: no contribution */
          add_JTJ(xs, h2 * bd->kappa, H);
          add_JT(xs, yo, h2 * bd->kappa, r);
          /* explicit remainder f_e = f - kappa (y_j - y_i) (friction clamp), i side */
          contact_force(bd, yi, yj, f);
          for (int q = 0; q < 3; ++q) fe[q] = f[q] - bd->kappa * (yj[q] - yi[q]);
          add_JT(xs, fe, side ? -h2 : h2, r);
          continue;
        }
        if (bd->type == ORACLE_BOND_SLIDER) {
          /* ball joint between x_i and the foot point of j at iterate k: the i
           * end is drawn to the foot, the foot point of j to y_i */
          double xf[3], yf[3];
          slider_foot(qk, bd, xf, yf);
          if (side == 0) {
            add_JTJ(bd->xi, h2 * bd->kappa, H);
            add_JT(bd->xi, yf, h2 * bd->kappa, r);
          } else {
            double yi[3];
            end_point(qk, bd->i, bd->xi, yi);
            add_JTJ(xf, h2 * bd->kappa, H);
            add_JT(xf, yi, h2 * bd->kappa, r);
          }
          continue;
        }
        if (bd->type == ORACLE_BOND_POLYNOMIAL) {
          double dv[3] = {yo[0] - ys[0], yo[1] - ys[1], yo[2] - ys[2]};
          double d = v3_norm(dv), w, phim;
          pabd_oracle_poly_split(bd->kappa, bd->order, bd->rest, d, &w, &phim);
          add_JTJ(xs, h2 * w, H);
          add_JT(xs, yo, h2 * w, r);
          if (d > 1e-12 && phim != 0.0) {
            double nrm[3] = {dv[0] / d, dv[1] / d, dv[2] / d};
            add_JT(xs, nrm, h2 * phim, r);
          }
          continue;
        }
        if (bd->type == ORACLE_BOND_AUGMENTED) {
          /* Psi = 1/2 kappa C^2 + lambda C with the signed elongation C = d - l
           * (reading): phi = dPsi/dd = kappa d + (lambda - kappa l), split by the
           * rule of Sec. 4.2.1 (phi^+ >= 0 implicit, phi^- <= 0 explicit):
           * phi^+ = kappa d + max(lambda - kappa l, 0), i.e. the weight
           * w = kappa + (lambda - kappa l) / d^k while the remainder is a
           * tension, and phi^- = min(lambda - kappa l, 0) explicit along n */
          double dv[3] = {yo[0] - ys[0], yo[1] - ys[1], yo[2] - ys[2]};
          double d = v3_norm(dv);
          double phim = bd->al_lambda - bd->al_kappa * bd->rest;
          double w = bd->al_kappa;
          if (phim > 0.0 && d > 1e-12) {
            w += phim / d;
            phim = 0.0;
          }
          add_JTJ(xs, h2 * w, H);
          add_JT(xs, yo, h2 * w, r);
          if (d > 1e-12 && phim != 0.0) {
            double nrm[3] = {dv[0] / d, dv[1] / d, dv[2] / d};
            add_JT(xs, nrm, h2 * phim, r);
          }
          continue;
        }
        /* implicit part: h^2 phi^+(d)/d J^T y_j with phi^+/d = kappa */
        add_JTJ(xs, h2 * bd->kappa, H);
        add_JT(xs, yo, h2 * bd->kappa, r);
        if (bd->rest > 0.0) {
          /* explicit part h^2 phi^-(d) J^T n with phi^- = -kappa l (quadratic
           * spring split: phi = kappa (d - l) = kappa d + (-kappa l)) */
          double dv[3] = {yo[0] - ys[0], yo[1] - ys[1], yo[2] - ys[2]};
          double d = v3_norm(dv);
          if (d > 1e-12) {
            double nrm[3] = {dv[0] / d, dv[1] / d, dv[2] / d};
            add_JT(xs, nrm, h2 * (-bd->kappa * bd->rest), r);
          }
        }
      }
      double Lf[144], qh[12];
      memcpy(Lf, H, sizeof Lf);
      if (cholesky(Lf, 12) != 0) {
        status = -1;
        break;
      }
      cholesky_solve(Lf, 12, r, qh);
      memcpy(o->q_half + 12 * b, qh, sizeof qh);
      /* local solve: c unchanged, A <- rotation factor of A^{k+1/2} */
      memcpy(qnext + 12 * b, qh, 3 * sizeof(double));
      if (o->debug & 1)
        memcpy(qnext + 12 * b + 3, qh + 3, 9 * sizeof(double));
      else
        pabd_oracle_polar(qh + 3, qnext + 12 * b + 3);
      double dq[12];
      for (int a = 0; a < 12; ++a) dq[a] = qnext[12 * b + a] - qk[12 * b + a];
      num += m_norm2(o->mass[b], o->Pi + 9 * b, dq);
      den += m_norm2(o->mass[b], o->Pi + 9 * b, qk + 12 * b);
    }
    o->rho[k] = den > 0.0 ? sqrt(num / den) : 0.0;
    /* augmented bonds (Sec. 5.2.2): lambda^{k+1} = kappa^k C^k + lambda^k and
     * kappa^{k+1} = kappa^k + beta |C^k|, C^k taken above */
    for (int e = 0; e < o->n_static; ++e) {
      bond_t *bd = &o->bonds[e];
      if (bd->type != ORACLE_BOND_AUGMENTED) continue;
      bd->al_lambda = bd->al_kappa * al_C[e] + bd->al_lambda;
      bd->al_kappa = bd->al_kappa + o->al_beta * fabs(al_C[e]);
    }
    memcpy(o->q_prev, qk, (size_t)n * 12 * sizeof(double));
    double *tmp = qk;
    qk = qnext;
    qnext = tmp;
  }

  /* Algorithm 1: velocity recovery */
  for (int b = 0; b < n && status == 0; ++b) {
    if (pinned(o, b)) continue;
    double *cnew = qk + 12 * b, *Anew = qk + 12 * b + 3;
    for (int k = 0; k < 3; ++k) o->v[3 * b + k] = (cnew[k] - o->c[3 * b + k]) / h;
    double dA[9], Ainv[9], W[9];
    for (int k = 0; k < 9; ++k) dA[k] = Anew[k] - o->A[9 * b + k];
    if (m3_inverse(o->A + 9 * b, Ainv) != 0) {
      status = -1;
      break;
    }
    m3_mul(dA, Ainv, W);
    for (int k = 0; k < 9; ++k) W[k] /= h;
    /* average of [w]_x and -[w]_x^T, read off the off-diagonal entries */
    o->w[3 * b + 0] = 0.5 * (W[7] - W[5]);
    o->w[3 * b + 1] = 0.5 * (W[2] - W[6]);
    o->w[3 * b + 2] = 0.5 * (W[3] - W[1]);
    memcpy(o->c + 3 * b, cnew, 3 * sizeof(double));
    memcpy(o->A + 9 * b, Anew, 9 * sizeof(double));
  }
  for (int b = 0; b < n && status == 0; ++b)
    for (int k = 0; k < 3; ++k)
      if (!isfinite(o->c[3 * b + k]) || !isfinite(o->v[3 * b + k])) status = -1;
  free(al_C);
  for (int e = 0; e < o->n_static; ++e)
    if (o->bonds[e].type == ORACLE_BOND_AUGMENTED) {
      o->static_bonds[e].al_kappa = o->bonds[e].al_kappa;
      o->static_bonds[e].al_lambda = o->bonds[e].al_lambda;
    }
  free(s);
  free(qk);
  free(qnext);
  o->steps_done++;
  return status;
}

int pabd_oracle_step(pabd_oracle *o, int32_t nsteps) {
  for (int i = 0; i < nsteps; ++i)
    if (one_step(o) != 0) return -1;
  return 0;
}
