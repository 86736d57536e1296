// host_scene.h -- host-side preparation of one scene description: validation,
// per-body mass and affine moment (Sec. 4.1.1), bond-end incidence lists in
// (body, bond id) order, driven-bond table.  Everything here is FP64; upload
// converts to the scene's arithmetic type.
#pragma once

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/pabd.h"
#include "common.h"

namespace pabd {

struct HostScene {
  int n = 0, ne = 0;
  std::vector<double> qn, vel, mass64, half;  // 12, 8, 8, 4 per body
  std::vector<uint8_t> flags, shape;
  std::vector<int> group;
  std::vector<int> srow, se_partner;  // scene-local partner ids
  std::vector<double> se;             // 8 per end (FP64 master copy)
  std::vector<double> se64;           // 4 per end
  std::vector<double> al;             // 4 per end: augmented (kappa_j, lambda_j, l, kappa_start),
                                      // polynomial (kappa, 0, l, -p), else zeros
  std::vector<int> bond_end;          // scene-local end of every bond held by a free body (i side if free)
  std::vector<int> drv_end_i, drv_end_j;
  std::vector<double> drv_param;      // 13 per driven bond
  std::vector<double> planes;         // 4 per plane
  SceneDev params{};
  bool contact = false, driven = false, variable = false;
  int ccap = 0;
  int max_ends = 0;  // largest number of static ends of one body
};

inline double sqr(double x) { return x * x; }

// Returns an empty string on success, else the reason the description is invalid.
inline std::string build_host_scene(const pabd_scene_desc* d, HostScene& hs) {
  if (!d) return "null descriptor";
  if (d->n_bodies < 0 || d->n_bonds < 0) return "negative body or bond count";
  if (!(d->h > 0.0) || !std::isfinite(d->h)) return "time step h must be positive";
  if (d->iters < 1) return "iters must be >= 1";
  if (d->precision != PABD_FP32 && d->precision != PABD_FP64) return "unknown precision";
  const int n = d->n_bodies;
  if (n > 0 && (!d->shape || !d->shape_param || !d->c0 || !d->A0 || (!d->density && !(d->mass && d->Pi0))))
    return "missing body arrays";
  if (d->n_bonds > 0 && (!d->bond_i || !d->bond_j || !d->x_i || !d->x_j || !d->kappa))
    return "missing bond arrays";
  hs.n = n;
  hs.qn.assign(12 * (size_t)n, 0.0);
  hs.vel.assign(8 * (size_t)n, 0.0);
  hs.mass64.assign(8 * (size_t)n, 0.0);
  hs.half.assign(4 * (size_t)n, 0.0);
  hs.flags.assign(n, 0);
  hs.shape.assign(n, 0);
  hs.group.assign(n, 0);
  for (int b = 0; b < n; ++b) {
    const int sh = d->shape[b];
    if (sh != PABD_SHAPE_BOX && sh != PABD_SHAPE_SPHERE) return "unknown shape of body " + std::to_string(b);
    const double* p = d->shape_param + 3 * (size_t)b;
    const uint8_t fl = d->flags ? (uint8_t)(d->flags[b] & (PABD_FLAG_PINNED | PABD_FLAG_NO_CONTACT)) : 0;
    hs.flags[b] = fl;
    hs.shape[b] = (uint8_t)sh;
    hs.group[b] = d->group ? d->group[b] : 0;
    const double rho = d->density ? d->density[b] : 0.0;
    double m, P0, P1, P2;
    if (sh == PABD_SHAPE_BOX) {
      if (!(p[0] > 0 && p[1] > 0 && p[2] > 0)) return "box half extents must be positive";
      // int rho x x^T over [-hx,hx]x[-hy,hy]x[-hz,hz] = m diag(hx^2, hy^2, hz^2) / 3
      m = rho * 8.0 * p[0] * p[1] * p[2];
      P0 = m * p[0] * p[0] / 3.0;
      P1 = m * p[1] * p[1] / 3.0;
      P2 = m * p[2] * p[2] / 3.0;
      hs.half[4 * b] = p[0];
      hs.half[4 * b + 1] = p[1];
      hs.half[4 * b + 2] = p[2];
      hs.half[4 * b + 3] = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    } else {
      if (!(p[0] > 0)) return "sphere radius must be positive";
      // ball of radius r: m = rho 4 pi r^3 / 3, int rho x x^T = m r^2 / 5 I
      m = rho * 4.0 * M_PI * p[0] * p[0] * p[0] / 3.0;
      P0 = P1 = P2 = m * p[0] * p[0] / 5.0;
      for (int k = 0; k < 4; ++k) hs.half[4 * b + k] = p[0];
    }
    const bool pinned = (fl & PABD_FLAG_PINNED) != 0;
    // packed symmetric Pi0: 00 01 02 11 12 22; given, or the shape's principal moments
    double P[6] = {P0, 0.0, 0.0, P1, 0.0, P2};
    if (d->mass) m = d->mass[b];
    if (d->Pi0)
      for (int k = 0; k < 6; ++k) P[k] = d->Pi0[6 * (size_t)b + k];
    if (!pinned) {
      if (!(m > 0.0 && std::isfinite(m))) return "free body " + std::to_string(b) + " needs positive mass";
      // Sylvester's criterion on the leading minors
      const double m1 = P[0], m2 = P[0] * P[3] - P[1] * P[1];
      const double m3 = P[0] * (P[3] * P[5] - P[4] * P[4]) - P[1] * (P[1] * P[5] - P[4] * P[2]) +
                        P[2] * (P[1] * P[4] - P[3] * P[2]);
      bool finite = true;
      for (double x : P) finite = finite && std::isfinite(x);
      if (!finite || !(m1 > 0.0 && m2 > 0.0 && m3 > 0.0))
        return "free body " + std::to_string(b) + " needs a symmetric positive definite Pi0";
    }
    double* M = &hs.mass64[8 * (size_t)b];
    M[0] = m; M[1] = P[0]; M[2] = P[1]; M[3] = P[2]; M[4] = P[3]; M[5] = P[4]; M[6] = P[5]; M[7] = 0;
    for (int k = 0; k < 3; ++k) hs.qn[12 * b + k] = d->c0[3 * b + k];
    for (int k = 0; k < 9; ++k) hs.qn[12 * b + 3 + k] = d->A0[9 * b + k];
    if (!pinned) {
      for (int k = 0; k < 3; ++k) {
        hs.vel[8 * b + k] = d->v0 ? d->v0[3 * b + k] : 0.0;
        hs.vel[8 * b + 3 + k] = d->w0 ? d->w0[3 * b + k] : 0.0;
      }
    }
    for (int k = 0; k < 12; ++k)
      if (!std::isfinite(hs.qn[12 * b + k])) return "non-finite initial state";
    // A0 must be a rotation: the prediction turns it by R(dQ) and the velocity
    // recovery inverts it by its transpose
    const double* A = d->A0 + 9 * (size_t)b;
    double e2 = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const double g = A[r] * A[c] + A[3 + r] * A[3 + c] + A[6 + r] * A[6 + c] - (r == c ? 1.0 : 0.0);
        e2 += g * g;
      }
    const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                       A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(e2 <= 1e-12 && det > 0.0)) return "A0 of body " + std::to_string(b) + " is not a rotation";
  }
  // bond ends, counting sort by owner keeping bond order (i side before j side)
  const int B = d->n_bonds;
  std::vector<int> cnt(n + 1, 0);
  int n_driven = 0;
  for (int e = 0; e < B; ++e) {
    const int i = d->bond_i[e], j = d->bond_j[e];
    const int ty = d->bond_type ? d->bond_type[e] : PABD_BOND_QUADRATIC;
    if (i < 0 || i >= n || j < -1 || j >= n || i == j) return "bond " + std::to_string(e) + " has bad endpoints";
    if (ty != PABD_BOND_QUADRATIC && ty != PABD_BOND_DRIVEN && ty != PABD_BOND_AUGMENTED &&
        ty != PABD_BOND_POLYNOMIAL && ty != PABD_BOND_SLIDER)
      return "unknown bond type";
    if (ty == PABD_BOND_SLIDER) {
      if (!d->drive) return "slider bond without its axis (drive[0..2])";
      const double* u = d->drive + 13 * (size_t)e;
      const double un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      if (!(un > 0.0) || !std::isfinite(un)) return "slider axis must be finite and nonzero";
      if (d->rest_len && d->rest_len[e] != 0.0) return "slider bond needs rest length 0";
    }
    if (ty == PABD_BOND_POLYNOMIAL) {
      const int p = d->order ? d->order[e] : 0;
      if (p < 2 || p > 12 || p % 2 != 0) return "polynomial bond order must be even in [2, 12]";
    }
    if (!(d->kappa[e] > 0.0)) return "bond stiffness must be positive";
    if (d->rest_len && d->rest_len[e] < 0.0) return "rest length must be >= 0";
    if (ty == PABD_BOND_AUGMENTED) {
      // with l = 0 the elongation d >= 0 never changes sign: the multiplier could only grow
      if (!d->rest_len || !(d->rest_len[e] > 0.0)) return "augmented bond needs a rest length > 0";
      if (!(d->al_beta >= 0.0 && d->al_alpha >= 0.0 && d->al_gamma >= 0.0))
        return "augmented-bond constants must be >= 0";
    }
    if (ty == PABD_BOND_DRIVEN) {
      if (!d->drive) return "driven bond without drive parameters";
      ++n_driven;
    }
    cnt[i + 1]++;
    if (j >= 0) cnt[j + 1]++;
  }
  hs.srow.assign(n + 1, 0);
  for (int b = 0; b < n; ++b) hs.srow[b + 1] = hs.srow[b] + cnt[b + 1];
  hs.ne = hs.srow[n];
  hs.se_partner.assign(hs.ne, -1);
  hs.se.assign(8 * (size_t)hs.ne, 0.0);
  hs.se64.assign(4 * (size_t)hs.ne, 0.0);
  hs.al.assign(4 * (size_t)hs.ne, 0.0);
  hs.bond_end.assign(B, -1);
  hs.variable = false;
  std::vector<int> fill(n, 0);
  hs.drv_end_i.clear();
  hs.drv_end_j.clear();
  hs.drv_param.clear();
  for (int e = 0; e < B; ++e) {
    const int i = d->bond_i[e], j = d->bond_j[e];
    const double kap = d->kappa[e], l = d->rest_len ? d->rest_len[e] : 0.0;
    const double* xi = d->x_i + 3 * (size_t)e;
    const double* xj = d->x_j + 3 * (size_t)e;
    const int ei = hs.srow[i] + fill[i]++;
    hs.bond_end[e] = ei;
    hs.se_partner[ei] = j;
    double* E = &hs.se[8 * (size_t)ei];
    E[0] = xi[0]; E[1] = xi[1]; E[2] = xi[2]; E[3] = kap;
    E[4] = xj[0]; E[5] = xj[1]; E[6] = xj[2]; E[7] = -kap * l;
    double* E64 = &hs.se64[4 * (size_t)ei];
    E64[0] = xi[0]; E64[1] = xi[1]; E64[2] = xi[2]; E64[3] = kap;
    int ej = -1;
    if (j >= 0) {
      ej = hs.srow[j] + fill[j]++;
      hs.se_partner[ej] = i;
      double* F = &hs.se[8 * (size_t)ej];
      F[0] = xj[0]; F[1] = xj[1]; F[2] = xj[2]; F[3] = kap;
      F[4] = xi[0]; F[5] = xi[1]; F[6] = xi[2]; F[7] = -kap * l;
      double* F64 = &hs.se64[4 * (size_t)ej];
      F64[0] = xj[0]; F64[1] = xj[1]; F64[2] = xj[2]; F64[3] = kap;
    }
    const int ty = d->bond_type ? d->bond_type[e] : PABD_BOND_QUADRATIC;
    if (ty == PABD_BOND_AUGMENTED || ty == PABD_BOND_POLYNOMIAL) {
      // per-end data (augmented: both ends keep identical copies of the state);
      // the weight changes every iteration, so the bond stays out of the static
      // block (se64 kappa 0)
      hs.variable = true;
      const bool aug = ty == PABD_BOND_AUGMENTED;
      for (int ee : {ei, ej}) {
        if (ee < 0) continue;
        double* a = &hs.al[4 * (size_t)ee];
        a[0] = kap;
        a[1] = 0.0;
        a[2] = l;
        a[3] = aug ? kap : -(double)d->order[e];
        hs.se64[4 * (size_t)ee + 3] = 0.0;
      }
      hs.flags[i] |= F_VARIABLE;
      if (j >= 0) hs.flags[j] |= F_VARIABLE;
      // a pinned body never iterates, so its copy of the state is not advanced
      if ((hs.flags[i] & PABD_FLAG_PINNED) && ej >= 0) hs.bond_end[e] = ej;
    }
    if (ty == PABD_BOND_SLIDER) {
      // per-end axis u (unit, line body's frame) and side code; the point side's
      // weight sits at its fixed anchor (static block), the line side's at the
      // foot, which moves every iteration (se64 kappa 0)
      hs.variable = true;
      const double* u = d->drive + 13 * (size_t)e;
      const double un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      for (int ee : {ei, ej}) {
        if (ee < 0) continue;
        double* a = &hs.al[4 * (size_t)ee];
        a[0] = u[0] / un;
        a[1] = u[1] / un;
        a[2] = u[2] / un;
        a[3] = ee == ei ? AL_SLIDER_POINT : AL_SLIDER_LINE;
      }
      if (ej >= 0) hs.se64[4 * (size_t)ej + 3] = 0.0;
      hs.flags[i] |= F_VARIABLE;
      if (j >= 0) hs.flags[j] |= F_VARIABLE;
    }
    if (ty == PABD_BOND_DRIVEN) {
      hs.drv_end_i.push_back(ei);
      hs.drv_end_j.push_back(ej);
      for (int k = 0; k < 13; ++k) hs.drv_param.push_back(d->drive[13 * (size_t)e + k]);
    }
  }
  hs.max_ends = 0;
  for (int b = 0; b < n; ++b) hs.max_ends = std::max(hs.max_ends, hs.srow[b + 1] - hs.srow[b]);
  hs.driven = n_driven > 0;
  hs.contact = d->contact_enable != 0;
  if (hs.contact) {
    if (d->max_contacts_per_body <= 0) return "contacts need max_contacts_per_body > 0";
    if (d->n_planes > 0 && !d->planes) return "missing planes";
  }
  hs.ccap = hs.contact ? d->max_contacts_per_body : 0;
  hs.planes.assign(d->planes ? d->planes : nullptr,
                   d->planes ? d->planes + 4 * (size_t)std::max(d->n_planes, 0) : nullptr);
  SceneDev& S = hs.params;
  S = SceneDev{};
  S.h = d->h;
  S.g0 = d->gravity[0];
  S.g1 = d->gravity[1];
  S.g2 = d->gravity[2];
  S.t0 = d->t0;
  S.kscale = d->contact_kappa_scale;
  S.margin = d->contact_margin;
  S.mu = d->mu;
  S.cell = 1.0;
  S.iters = d->iters;
  S.n_bodies = n;
  S.n_planes = hs.contact ? std::max(d->n_planes, 0) : 0;
  S.contact = hs.contact ? 1 : 0;
  S.ccap = hs.ccap;
  S.al_beta = d->al_beta;
  S.al_alpha = d->al_alpha;
  S.al_gamma = d->al_gamma;
  return "";
}

// device bytes of one scene at arithmetic type size ts (admission bound)
inline size_t scene_bytes(const HostScene& hs, int ts) {
  const size_t per_body = (size_t)ts * (4 * (QW + 4) + VW + MW + FW + 4) + 8 * (10 + 8 + 2) + 2 + 4 * 4;
  const size_t per_end = (size_t)ts * (EW + 4) + 4 + 8 * 4;
  // contact slots (final and staging) and the broad phase: record, reach,
  // large-list entry and task offset, and max(16, ccap / 2) candidate pairs per body
  // final record, partner and key, then the staged copy
  const size_t per_contact = (size_t)ts * (ts == 4 ? ContactRec<float>::W : ContactRec<double>::W) + 4 + 8 +
                             (ts == 4 ? sizeof(StageRec<float>) : sizeof(StageRec<double>));
  const size_t per_contact_body = hs.ccap > 0 ? 64 + 8 + 4 + 4 + 8 * (size_t)std::max(16, hs.ccap / 2) : 0;
  return per_body * hs.n + per_end * hs.ne + per_contact * (size_t)hs.n * hs.ccap +
         per_contact_body * hs.n +
         hs.drv_param.size() * 8 + hs.planes.size() * 8 + sizeof(SceneDev) + 64;
}

}  // namespace pabd
