// kernels_contact.h -- contact-bond construction (collision detection of
// Algorithm 1) on q^n, for every scene with contacts enabled.
//
// Reading of the contact bond (the paper gives its contact and friction energies
// only in a supplement): a contact joins a point x_i of body i (a box vertex or a
// sphere surface point) to the closest surface point x_j of body j (material frame
// of j, or world coordinates for a plane), with a unit normal n fixed for the
// step (outward from j, towards i) and stiffness kappa_c = scale * m / h^2, m the
// heavier free mass of the pair.  Detection uses a speculative margin
// pm = margin + h (|v| + |w| R) per body (R: bounding radius; spheres omit
// the spin term).
//
// Pipeline: k_contact_prep (margins, per-scene max reach, clear counters) ->
// k_hash_count / scan / k_hash_fill (uniform grid of cell 2 max(R + pm), spatial
// hash with scene id) -> k_narrow (27 neighbour cells, each pair once by its
// lower index, plus planes) -> k_sort_contacts (per-body canonical order, so the
// iteration sums in a fixed order whatever order the atomics produced).
#pragma once

#include "common.h"
#include "device_math.h"

namespace pabd {

struct ContactBuf {
  int tb;                // hash buckets (power of two)
  int* bucket_count;     // [tb]
  int* bucket_start;     // [tb + 1]
  int* bucket_fill;      // [tb]
  int* sorted_body;      // [n]
  unsigned long long* reach;  // per scene: max(R + pm) as double bits
  const double* mass64;  // 8 per body
  int* scan_tmp;         // block sums
};

// speculative margin: the body's surface moves by about h (|v| + |w| R) in a
// step; spheres omit the spin term (spinning does not move their surface)
__device__ __forceinline__ double body_pm(const SceneDev& S, const double* vw, double R, int shape) {
  double vn = sqrt(vw[0] * vw[0] + vw[1] * vw[1] + vw[2] * vw[2]);
  double wn = shape == 0 ? sqrt(vw[3] * vw[3] + vw[4] * vw[4] + vw[5] * vw[5]) * R : 0.0;
  return S.margin + S.h * (vn + wn);
}

template <typename T>
__device__ __forceinline__ bool contact_body(const View<T>& v, int i, int sc) {
  return sc >= 0 && v.scenes[sc].contact && v.scenes[sc].step < v.scenes[sc].steps_total &&
         !(v.flags[i] & F_NOCONTACT);
}

template <typename T>
__global__ void k_contact_prep(View<T> v, ContactBuf cb, int n_scenes) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_scenes) cb.reach[i] = 0ull;
  if (i >= v.n) return;
  v.ccount[i] = 0;
  v.r_num[i] = 0.0;
  v.r_den[i] = 0.0;
}

template <typename T>
__global__ void k_contact_reach(View<T> v, ContactBuf cb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.n) return;
  const int sc = v.bscene[i];
  if (!contact_body(v, i, sc)) return;
  T vw[VW];
  load<T, VW>(v.vel + (size_t)VW * i, vw);
  double vd[6] = {(double)vw[0], (double)vw[1], (double)vw[2], (double)vw[3], (double)vw[4], (double)vw[5]};
  double R = (double)v.half[4 * i + 3];
  double reach = R + body_pm(v.scenes[sc], vd, R, v.shape[i]);
  atomicMax(cb.reach + sc, (unsigned long long)__double_as_longlong(reach));
}

__global__ void k_contact_cells(SceneDev* scenes, int n_scenes, const unsigned long long* reach) {
  const int sc = blockIdx.x * blockDim.x + threadIdx.x;
  if (sc >= n_scenes) return;
  double r = __longlong_as_double((long long)reach[sc]);
  scenes[sc].cell = r > 0.0 ? 2.0 * r : 1.0;
}

__device__ __forceinline__ unsigned bucket_of(int sc, int cx, int cy, int cz, int tb) {
  unsigned h = (unsigned)cx * 73856093u ^ (unsigned)cy * 19349663u ^ (unsigned)cz * 83492791u ^
               (unsigned)sc * 2654435761u;
  h ^= h >> 13;
  h *= 0x5bd1e995u;
  h ^= h >> 15;
  return h & (unsigned)(tb - 1);
}

template <typename T>
__device__ __forceinline__ void cell_of(const View<T>& v, int i, double cell, int* cc) {
  const T* q = v.qn + (size_t)Rec<T>::Q * i;
  cc[0] = (int)floor(pos_value(q, 0) / cell);
  cc[1] = (int)floor(pos_value(q, 1) / cell);
  cc[2] = (int)floor(pos_value(q, 2) / cell);
}

__global__ void k_zero_int(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <typename T>
__global__ void k_hash_count(View<T> v, ContactBuf cb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.n) return;
  const int sc = v.bscene[i];
  if (!contact_body(v, i, sc)) return;
  int cc[3];
  cell_of(v, i, v.scenes[sc].cell, cc);
  atomicAdd(cb.bucket_count + bucket_of(sc, cc[0], cc[1], cc[2], cb.tb), 1);
}

template <typename T>
__global__ void k_hash_fill(View<T> v, ContactBuf cb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.n) return;
  const int sc = v.bscene[i];
  if (!contact_body(v, i, sc)) return;
  int cc[3];
  cell_of(v, i, v.scenes[sc].cell, cc);
  unsigned b = bucket_of(sc, cc[0], cc[1], cc[2], cb.tb);
  int pos = atomicAdd(cb.bucket_fill + b, 1);
  cb.sorted_body[cb.bucket_start[b] + pos] = i;
}

// ---- exclusive scan of int counts (three passes, 1024 per block) ---------------

__global__ void __launch_bounds__(1024) k_scan_block(const int* in, int* out, int n, int* block_sums) {
  __shared__ int sh[1024];
  const int t = threadIdx.x, i = blockIdx.x * 1024 + t;
  int x = i < n ? in[i] : 0;
  sh[t] = x;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int y = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += y;
    __syncthreads();
  }
  if (i < n) out[i] = sh[t] - x;
  if (t == 1023) block_sums[blockIdx.x] = sh[1023];
}

__global__ void __launch_bounds__(1024) k_scan_sums(int* block_sums, int nb, int* total_out) {
  __shared__ int sh[1024];
  const int t = threadIdx.x;
  int x = t < nb ? block_sums[t] : 0;
  sh[t] = x;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int y = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += y;
    __syncthreads();
  }
  if (t < nb) block_sums[t] = sh[t] - x;
  if (t == 1023) *total_out = sh[1023];
}

__global__ void k_scan_add(int* out, int n, const int* block_sums) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += block_sums[i / 1024];
}

// ---- narrow phase ----------------------------------------------------------------

template <typename T>
struct Narrow {
  View<T> v;
  ContactBuf cb;
};

template <typename T>
__device__ __forceinline__ double free_mass(const View<T>& v, const ContactBuf& cb, int b) {
  if (b < 0 || (v.flags[b] & F_PINNED)) return 0.0;
  return cb.mass64[8 * (size_t)b];
}

// write one bond end into the owner's slot list
template <typename T>
__device__ __forceinline__ void push_end(const View<T>& v, int owner, int sc, int partner,
                                         int feature, int side, const double* xs,
                                         const double* xo, const double* n, double kap,
                                         double mu) {
  const int cap = v.scenes[sc].ccap;
  const int slot = atomicAdd(v.ccount + owner, 1);
  if (slot >= cap) {
    atomicOr(v.health + sc, 2);
    return;
  }
  const size_t e = (size_t)owner * cap + slot;
  T C[CW] = {(T)xs[0], (T)xs[1], (T)xs[2], (T)kap, (T)xo[0], (T)xo[1], (T)xo[2], (T)mu,
             (T)n[0], (T)n[1], (T)n[2], (T)0};
  store<T, CW>(v.ce + CW * e, C);
  v.ce_partner[e] = partner;
  v.ce_key[e] = ((unsigned long long)(unsigned)(partner + 1) << 32) |
                ((unsigned long long)(unsigned)feature << 1) | (unsigned)side;
}

template <typename T>
__device__ __forceinline__ void emit_contact(const View<T>& v, const ContactBuf& cb, int sc,
                                             int i, int j, int feature, const double* xi,
                                             const double* xj, const double* n) {
  const SceneDev& S = v.scenes[sc];
  double m = fmax(free_mass(v, cb, i), free_mass(v, cb, j));
  double kap = S.kscale * m / (S.h * S.h);
  push_end(v, i, sc, j, feature, 0, xi, xj, n, kap, S.mu);
  if (j >= 0) {
    double nn[3] = {-n[0], -n[1], -n[2]};
    push_end(v, j, sc, i, feature, 1, xj, xi, nn, kap, S.mu);
  }
}

template <typename T>
struct BodyGeo {
  double c[3], A[9], he[3], R;
  int shape;
};

template <typename T>
__device__ __forceinline__ void body_geo(const View<T>& v, int b, BodyGeo<T>& g) {
  const T* q = v.qn + (size_t)Rec<T>::Q * b;
  for (int k = 0; k < 3; ++k) g.c[k] = pos_value(q, k);
  for (int k = 0; k < 9; ++k) g.A[k] = (double)q[3 + k];
  for (int k = 0; k < 3; ++k) g.he[k] = (double)v.half[4 * b + k];
  g.R = (double)v.half[4 * b + 3];
  g.shape = v.shape[b];
}

__device__ __forceinline__ void vertex_of(int k, const double* he, double* x) {
  x[0] = (k & 1) ? he[0] : -he[0];
  x[1] = (k & 2) ? he[1] : -he[1];
  x[2] = (k & 4) ? he[2] : -he[2];
}

// box-box, vertex-face: reference face = face axis (3 of i, then 3 of j) of least
// overlap; incident vertices within the margin of that face and inside its
// lateral extent become contacts (incident box = i side, reference box = j side)
template <typename T>
__device__ void narrow_box_box(const View<T>& v, const ContactBuf& cb, int sc, int bi, int bj,
                               const BodyGeo<T>& gi, const BodyGeo<T>& gj, double pm) {
  const double dc[3] = {gj.c[0] - gi.c[0], gj.c[1] - gi.c[1], gj.c[2] - gi.c[2]};
  int best = -1;
  double best_ov = 0.0;
  for (int ax = 0; ax < 6; ++ax) {
    const double* A = ax < 3 ? gi.A : gj.A;
    const int k = ax % 3;
    const double u[3] = {A[k], A[3 + k], A[6 + k]};
    double ri = 0.0, rj = 0.0;
    for (int m = 0; m < 3; ++m) {
      ri += gi.he[m] * fabs(u[0] * gi.A[m] + u[1] * gi.A[3 + m] + u[2] * gi.A[6 + m]);
      rj += gj.he[m] * fabs(u[0] * gj.A[m] + u[1] * gj.A[3 + m] + u[2] * gj.A[6 + m]);
    }
    double ov = ri + rj - fabs(u[0] * dc[0] + u[1] * dc[1] + u[2] * dc[2]);
    if (ov < -pm) return;
    if (best < 0 || ov < best_ov) {
      best = ax;
      best_ov = ov;
    }
  }
  const bool ref_is_i = best < 3;
  const BodyGeo<T>& R = ref_is_i ? gi : gj;
  const BodyGeo<T>& I = ref_is_i ? gj : gi;
  const int ref = ref_is_i ? bi : bj, inc = ref_is_i ? bj : bi;
  const int k = best % 3;
  const double ax[3] = {R.A[k], R.A[3 + k], R.A[6 + k]};
  const double tw = ax[0] * (I.c[0] - R.c[0]) + ax[1] * (I.c[1] - R.c[1]) + ax[2] * (I.c[2] - R.c[2]);
  const double sgn = tw >= 0.0 ? 1.0 : -1.0;
  const double nw[3] = {sgn * ax[0], sgn * ax[1], sgn * ax[2]};
  for (int vtx = 0; vtx < 8; ++vtx) {
    double xv[3], p[3], rel[3], pl[3];
    vertex_of(vtx, I.he, xv);
    mat_vec(I.A, xv, p);
    for (int r = 0; r < 3; ++r) rel[r] = p[r] + I.c[r] - R.c[r];
    mat_tvec(R.A, rel, pl);
    const double gap = sgn * pl[k] - R.he[k];
    if (!(gap < pm) || gap < -2.0 * R.he[k]) continue;
    bool lateral = true;
    for (int m = 0; m < 3; ++m)
      if (m != k && fabs(pl[m]) > R.he[m] + pm) lateral = false;
    if (!lateral) continue;
    double xs[3];
    for (int m = 0; m < 3; ++m) xs[m] = pl[m] < -R.he[m] ? -R.he[m] : (pl[m] > R.he[m] ? R.he[m] : pl[m]);
    xs[k] = sgn * R.he[k];
    emit_contact(v, cb, sc, inc, ref, vtx, xv, xs, nw);
  }
}

// sphere s (i side) against box b (j side)
template <typename T>
__device__ void narrow_sphere_box(const View<T>& v, const ContactBuf& cb, int sc, int s, int b,
                                  const BodyGeo<T>& gs, const BodyGeo<T>& gb, double pm) {
  const double r = gs.he[0];
  double rel[3] = {gs.c[0] - gb.c[0], gs.c[1] - gb.c[1], gs.c[2] - gb.c[2]}, pl[3], q[3], nl[3];
  mat_tvec(gb.A, rel, pl);
  bool inside = true;
  for (int k = 0; k < 3; ++k) {
    q[k] = pl[k] < -gb.he[k] ? -gb.he[k] : (pl[k] > gb.he[k] ? gb.he[k] : pl[k]);
    if (q[k] != pl[k]) inside = false;
  }
  double gap;
  if (inside) {
    int ks = 0;
    double bestd = gb.he[0] - fabs(pl[0]);
    for (int k = 1; k < 3; ++k)
      if (gb.he[k] - fabs(pl[k]) < bestd) {
        bestd = gb.he[k] - fabs(pl[k]);
        ks = k;
      }
    const double sg = pl[ks] >= 0.0 ? 1.0 : -1.0;
    q[ks] = sg * gb.he[ks];
    nl[0] = nl[1] = nl[2] = 0.0;
    nl[ks] = sg;
    gap = -bestd - r;
  } else {
    const double dl[3] = {pl[0] - q[0], pl[1] - q[1], pl[2] - q[2]};
    const double dist = sqrt(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
    if (dist == 0.0) return;
    for (int k = 0; k < 3; ++k) nl[k] = dl[k] / dist;
    gap = dist - r;
  }
  if (!(gap < pm)) return;
  double nw[3], pw[3], xi[3];
  mat_vec(gb.A, nl, nw);
  for (int k = 0; k < 3; ++k) pw[k] = -r * nw[k];
  mat_tvec(gs.A, pw, xi);
  emit_contact(v, cb, sc, s, b, 8, xi, q, nw);
}

template <typename T>
__device__ void narrow_pair(const View<T>& v, const ContactBuf& cb, int sc, int i, int j,
                            const BodyGeo<T>& gi, double pmi) {
  BodyGeo<T> gj;
  body_geo(v, j, gj);
  T vw[VW];
  load<T, VW>(v.vel + (size_t)VW * j, vw);
  const double vd[6] = {(double)vw[0], (double)vw[1], (double)vw[2], (double)vw[3], (double)vw[4], (double)vw[5]};
  const double pm = pmi + body_pm(v.scenes[sc], vd, gj.R, gj.shape);
  const double dc[3] = {gj.c[0] - gi.c[0], gj.c[1] - gi.c[1], gj.c[2] - gi.c[2]};
  const double dist = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
  if (!(dist < gi.R + gj.R + pm)) return;
  if (gi.shape == 0 && gj.shape == 0) {
    narrow_box_box(v, cb, sc, i, j, gi, gj, pm);
  } else if (gi.shape == 1 && gj.shape == 1) {
    const double gap = dist - gi.he[0] - gj.he[0];
    if (!(gap < pm) || dist == 0.0) return;
    const double n[3] = {-dc[0] / dist, -dc[1] / dist, -dc[2] / dist};
    double pi_[3], pj[3], xi[3], xj[3];
    for (int k = 0; k < 3; ++k) {
      pi_[k] = -gi.he[0] * n[k];
      pj[k] = gj.he[0] * n[k];
    }
    mat_tvec(gi.A, pi_, xi);
    mat_tvec(gj.A, pj, xj);
    emit_contact(v, cb, sc, i, j, 8, xi, xj, n);
  } else if (gi.shape == 1) {
    narrow_sphere_box(v, cb, sc, i, j, gi, gj, pm);
  } else {
    narrow_sphere_box(v, cb, sc, j, i, gj, gi, pm);
  }
}

template <typename T>
__global__ void __launch_bounds__(128) k_narrow(View<T> v, ContactBuf cb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.n) return;
  const int sc = v.bscene[i];
  if (!contact_body(v, i, sc)) return;
  const SceneDev& S = v.scenes[sc];
  BodyGeo<T> gi;
  body_geo(v, i, gi);
  T vw[VW];
  load<T, VW>(v.vel + (size_t)VW * i, vw);
  const double vd[6] = {(double)vw[0], (double)vw[1], (double)vw[2], (double)vw[3], (double)vw[4], (double)vw[5]};
  const double pmi = body_pm(S, vd, gi.R, gi.shape);
  const bool pin_i = (v.flags[i] & F_PINNED) != 0;
  // planes
  if (!pin_i) {
    for (int p = 0; p < S.n_planes; ++p) {
      const double* pl = v.planes + 4 * (size_t)(S.plane_off + p);
      const double n[3] = {pl[0], pl[1], pl[2]};
      if (gi.shape == 0) {
        for (int k = 0; k < 8; ++k) {
          double x[3], y[3];
          vertex_of(k, gi.he, x);
          mat_vec(gi.A, x, y);
          for (int r = 0; r < 3; ++r) y[r] += gi.c[r];
          const double gap = n[0] * y[0] + n[1] * y[1] + n[2] * y[2] - pl[3];
          if (gap < pmi) {
            const double xw[3] = {y[0] - gap * n[0], y[1] - gap * n[1], y[2] - gap * n[2]};
            emit_contact(v, cb, sc, i, -1, 16 * p + k, x, xw, n);
          }
        }
      } else {
        const double r = gi.he[0];
        const double gap = n[0] * gi.c[0] + n[1] * gi.c[1] + n[2] * gi.c[2] - r - pl[3];
        if (gap < pmi) {
          const double pw[3] = {-r * n[0], -r * n[1], -r * n[2]};
          double x[3];
          mat_tvec(gi.A, pw, x);
          const double xw[3] = {gi.c[0] - (r + gap) * n[0], gi.c[1] - (r + gap) * n[1],
                                gi.c[2] - (r + gap) * n[2]};
          emit_contact(v, cb, sc, i, -1, 16 * p + 8, x, xw, n);
        }
      }
    }
  }
  // neighbour cells (each distinct bucket once)
  int cc[3];
  cell_of(v, i, S.cell, cc);
  unsigned seen[27];
  int nseen = 0;
  const int gi_group = v.group[i];
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const unsigned b = bucket_of(sc, cc[0] + dx, cc[1] + dy, cc[2] + dz, cb.tb);
        bool dup = false;
        for (int t = 0; t < nseen; ++t) dup = dup || seen[t] == b;
        if (dup) continue;
        seen[nseen++] = b;
        const int e1 = cb.bucket_start[b + 1];
        for (int e = cb.bucket_start[b]; e < e1; ++e) {
          const int j = cb.sorted_body[e];
          if (j <= i || v.bscene[j] != sc) continue;
          if (v.flags[j] & F_NOCONTACT) continue;
          if (pin_i && (v.flags[j] & F_PINNED)) continue;
          if (gi_group != 0 && v.group[j] == gi_group) continue;
          narrow_pair(v, cb, sc, i, j, gi, pmi);
        }
      }
}

// insertion sort of each body's contact ends by key
template <typename T>
__global__ void k_sort_contacts(View<T> v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.n) return;
  const int sc = v.bscene[i];
  if (!contact_body(v, i, sc)) return;
  const int cap = v.scenes[sc].ccap;
  int cnt = v.ccount[i];
  if (cnt > cap) cnt = cap;
  const size_t base = (size_t)i * cap;
  for (int a = 1; a < cnt; ++a) {
    unsigned long long key = v.ce_key[base + a];
    int b = a - 1;
    if (v.ce_key[base + b] <= key) continue;
    T C[CW];
    load<T, CW>(v.ce + CW * (base + a), C);
    const int part = v.ce_partner[base + a];
    while (b >= 0 && v.ce_key[base + b] > key) {
      v.ce_key[base + b + 1] = v.ce_key[base + b];
      v.ce_partner[base + b + 1] = v.ce_partner[base + b];
      T D[CW];
      load<T, CW>(v.ce + CW * (base + b), D);
      store<T, CW>(v.ce + CW * (base + b + 1), D);
      --b;
    }
    v.ce_key[base + b + 1] = key;
    v.ce_partner[base + b + 1] = part;
    store<T, CW>(v.ce + CW * (base + b + 1), C);
  }
}

}  // namespace pabd
