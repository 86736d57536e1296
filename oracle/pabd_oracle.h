/*
 * pabd_oracle.h -- interface of the plain FP64 CPU oracle for projective affine
 * body dynamics (PABD).
 *
 * TEST INFRASTRUCTURE ONLY.  The oracle exists to check the HIP library; it is
 * called by the test suite, by the package smoke check and by the CPU-baseline
 * leg of the benchmark, and by nothing else.  It shares no source, header,
 * helper or table with the HIP library (include/pabd.h is a different header
 * with different types), and it never calls the library.
 *
 * Everything is double precision, row-major, SI units.  All arrays passed in are
 * owned by the caller and copied at create time.
 *
 * Parity unpinned: the contact and friction model (contact bond, normal gate,
 * Coulomb clamp, stiffness and margin) is a reading of material the paper does
 * not print; it is held to the geometry and invariants of that reading
 * (closed-form contact points and normals, resting gaps, incline stick and
 * slip), not to the paper's own model.  The driven joint is a reading as well
 * (Sec. 5.3.3 gives a periodic target angle, not the joint's energy); it is
 * pinned against a ball joint to the target point turned by an independent
 * rotation routine.
 */
#ifndef PABD_ORACLE_H
#define PABD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* body shape ids */
#define ORACLE_SHAPE_BOX 0    /* shape_param = half extents (3) */
#define ORACLE_SHAPE_SPHERE 1 /* shape_param[0] = radius       */

/* body flag bits */
#define ORACLE_FLAG_PINNED 1u     /* kinematic: infinite mass, never updated */
#define ORACLE_FLAG_NO_CONTACT 2u /* excluded from collision detection       */

/* bond kinds */
#define ORACLE_BOND_QUADRATIC 0 /* Psi = 1/2 kappa (d - l)^2 (l = 0: ball joint) */
#define ORACLE_BOND_DRIVEN 1    /* ball joint whose j-side anchor follows a target angle */
#define ORACLE_BOND_CONTACT 2   /* created per step by collision detection      */
/* augmented Lagrangian (Sec. 5.2.2): Psi = 1/2 kappa_j C^2 + lambda_j C with the
 * signed elongation C = d - l (l > 0 required), kappa_j and lambda_j updated every
 * iteration and warm-started every step; the bond's kappa is kappa_start */
#define ORACLE_BOND_AUGMENTED 3
/* polynomial bond: Psi = kappa / p (d - l)^p, p even >= 2 (order[] of the bond);
 * phi = kappa (d - l)^{p-1} split by the sign of its binomial terms */
#define ORACLE_BOND_POLYNOMIAL 4
/* slider (point-on-line) bond, a reading: Sec. 5.1 names slider joints but gives
 * no energy.  Psi = 1/2 kappa dist(y_i, L_j)^2, where L_j is the line through
 * x_j along the unit axis u (both in j's material frame, world if j = -1; u is
 * drive[0..2] of the bond, rest_len must be 0).  Every iteration the line-side
 * anchor is the foot of the perpendicular from y_i^k onto L_j at q^k, and the
 * bond then acts as a ball joint between x_i and that material point of j */
#define ORACLE_BOND_SLIDER 5

typedef struct {
  int32_t n_bodies;
  const int32_t *shape;        /* [N] */
  const double *shape_param;   /* [N*3] */
  const double *density;       /* [N] kg/m^3 */
  const uint8_t *flags;        /* [N] */
  const int32_t *group;        /* [N] bodies sharing a nonzero group never collide */
  const double *c0, *A0;       /* [N*3], [N*9] */
  const double *v0, *w0;       /* [N*3], [N*3] */
  int32_t n_bonds;
  const int32_t *bond_i, *bond_j; /* [B]; j = -1: world anchor */
  const int32_t *bond_type;       /* [B] ORACLE_BOND_*, or NULL (all quadratic) */
  const double *x_i, *x_j;        /* [B*3] material anchors (world coords if j = -1) */
  const double *kappa, *rest_len; /* [B] */
  const double *drive;            /* [B*13]: axis(3) pivot(3) base(3) theta0 amp freq phase;
                                   * SLIDER bonds use axis(3) only */
  double gravity[3];
  double h;
  double t0; /* simulation time at the start of the first step */
  int32_t iters;
  int32_t contact_enable;
  double mu;
  double contact_kappa_scale; /* kappa_c = scale * m_max / h^2 (heavier free body) */
  double contact_margin;      /* base detection margin (m) */
  int32_t n_planes;
  const double *planes; /* [P*4]: unit normal n, offset o; free side n.y >= o */
  /* augmented-Lagrangian constants: stiffness growth beta, warm-start factors
   * alpha (multiplier) and gamma (both) */
  double al_beta, al_alpha, al_gamma;
  const int32_t *order; /* [B] polynomial order p of POLYNOMIAL bonds, or NULL */
  /* optional mass [N] and affine moment Pi0 [N*6] (packed symmetric 00 01 02 11
   * 12 22, material frame) of each body, replacing what density and shape give
   * (Sec. 4.1.1); NULL: from density and shape */
  const double *mass;
  const double *Pi0;
} pabd_oracle_desc;

typedef struct pabd_oracle pabd_oracle;

/* create / destroy; create returns NULL on an invalid descriptor (among others:
 * an A0 that is not a rotation, or a free body whose mass is not positive or
 * whose Pi0 is not positive definite) */
pabd_oracle *pabd_oracle_create(const pabd_oracle_desc *d);
void pabd_oracle_destroy(pabd_oracle *o);

/* advance nsteps steps of Algorithm 1; returns 0, or -1 on non-finite state */
int pabd_oracle_step(pabd_oracle *o, int32_t nsteps);

/* state read-back (any pointer may be NULL) */
void pabd_oracle_read_state(const pabd_oracle *o, double *c, double *A, double *v, double *w);

/* convergence residual rho_k of every iteration of the last step; returns K */
int pabd_oracle_residuals(const pabd_oracle *o, double *rho, int32_t cap);

/* debug switches: bit0 = skip the local (rigidification) step */
void pabd_oracle_set_debug(pabd_oracle *o, int32_t flags);

/* iterates of the last step: q^{K-1} (after projection) and q^{K-1/2}
 * (global result of the last iteration, before projection); [N*12] each */
void pabd_oracle_last_iterates(const pabd_oracle *o, double *q_prev, double *q_half);

/* mass and affine moment Pi0 (3x3) of one body shape at unit-free density */
void pabd_oracle_body_mass(int32_t shape, const double *param, double density, double *m,
                           double *Pi0);

/* nearest rotation of A (polar factor with determinant fix), via an SVD */
void pabd_oracle_polar(const double *A, double *R);

/* dense 12x12 H_i^k of body i at the last iteration of the last step */
void pabd_oracle_dense_H(const pabd_oracle *o, int32_t body, double *H);

/* contact bonds built by the last step's collision detection.
 * Returns their count; fills up to cap entries of each non-NULL array. */
int pabd_oracle_contacts(const pabd_oracle *o, int32_t cap, int32_t *ci, int32_t *cj,
                         int32_t *feature, double *xi, double *xj, double *normal,
                         double *kappa);

/* augmented-Lagrangian state of every bond after the last step (kappa_j, lambda_j;
 * kappa unchanged and lambda 0 for other kinds); any pointer may be NULL */
void pabd_oracle_bond_state(const pabd_oracle *o, double *kappa, double *lambda);

/* split of a polynomial bond's phi = kappa (d - l)^{p-1}: implicit weight
 * phi^+ / d and explicit phi^- (so w d + phim = phi, w >= 0, phim <= 0) */
void pabd_oracle_poly_split(double kappa, int32_t p, double l, double d, double *wplus,
                            double *phim);

/* build the contact set of the current state without stepping (same rule) */
int pabd_oracle_detect(pabd_oracle *o);

/* only the contacts that involve one body (its planes and its pairs), same rule;
 * replaces the stored contact set; -1 for a bad index */
int pabd_oracle_detect_body(pabd_oracle *o, int32_t body);

#ifdef __cplusplus
}
#endif

#endif
