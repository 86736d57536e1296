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
// Pipeline (one launch each):
//   k_contact_prep   clear per-body and per-scene counters (and the hash's
//                    bucket counts, when the step builds the hash); in the
//                    flat path also the step's prediction
//   k_contact_reach  reach = R + pm per body; per-scene maximum and a log-scale
//                    histogram of reach (four bins per octave)
//   k_contact_cells  per scene: cell = 2 cut, cut = the smaller of the maximum
//                    reach and the upper edge of the bin holding the 98th
//                    percentile; bodies with reach > cut are "large"
//   k_hash_count / scan / k_hash_fill   uniform-grid spatial hash of the small
//                    bodies (scene id in the hash), each bucket a run of 64-byte
//                    records holding the body's centre, reach, cell and filters;
//                    large bodies go to a list instead
//   k_broad_small    14 lanes per body: planes; then own cell and the 13 cells
//                    of the forward half-neighbourhood of a small body, one per
//                    lane, pairs with small bodies
//   k_large_tasks / k_broad_large   the large bodies' work in tasks of 256
//                    threads spread over the grid: small partners over the
//                    cells a body's reach spans (or over the scene's bodies when
//                    that is fewer), large partners of higher index
//   k_broad_brute    instead of the hash and both broad kernels, for a single
//                    scene of few bodies: one thread per pair
//   k_narrow_pairs   one thread per candidate pair: narrow phase, bond ends into
//                    the owners' staging slots
//   k_sort_contacts  one wave per body, ends copied in canonical key order to
//                    their final slots, so the iteration sums in a fixed order
//                    whatever order the atomics produced
// Candidate tests are conservative (a relative slack of 1e-12 on the sum of
// reaches); the narrow phase repeats the exact bounding test, so the contact
// set does not depend on the broad phase.
#pragma once

#include "common.h"
#include "contact_record.h"
#include "device_math.h"
#include "kernels_step.h"

namespace pabd {

// broad-phase record of a small body, in bucket order (32 bytes): centre and
// reach rounded to float (tests against them carry a slack that covers the
// rounding), body and scene, and the cell packed as three 21-bit fields
struct BroadRec {
  float c[3];
  float reach;
  int body, scene;
  unsigned long long cell;
};

__device__ __forceinline__ unsigned long long pack_cell(int x, int y, int z) {
  auto f = [](int a) {
    a = a < -(1 << 20) ? -(1 << 20) : (a > (1 << 20) - 1 ? (1 << 20) - 1 : a);
    return (unsigned long long)(unsigned)(a + (1 << 20));
  };
  return (f(x) << 42) | (f(y) << 21) | f(z);
}

constexpr int REACH_BINS = 64;
constexpr int REACH_BIN_BASE = 468;  // float bits >> 21 of 2^-10: bins span 2^-10 .. 2^6

struct ContactBuf {
  int tb;                // hash buckets (power of two)
  int* bucket_count;     // [tb]
  int* bucket_start;     // [tb + 1]
  int* bucket_fill;      // [tb]
  BroadRec* rec;         // [nc] small bodies in bucket order
  unsigned long long* reach;  // per scene: max(R + pm) as double bits
  int* hist;             // per scene: REACH_BINS counts
  double* breach;        // per body: R + pm
  int* large;            // [nc] large bodies
  int* counters;         // [0] large bodies, [1] candidate pairs, [2] large-body tasks
  int2* pairs;           // [pcap]
  int pcap;
  const double* mass64;  // 8 per body
  int* scan_tmp;         // block sums
  int* ltask;            // [nc + 1] first task of each large body (exclusive prefix)
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
__global__ void k_contact_prep(View<T> v, ContactBuf cb, int n_scenes, int n_buckets, bool predict) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_buckets) {  // the spatial hash's counts, when this step builds it
    cb.bucket_count[i] = 0;
    cb.bucket_fill[i] = 0;
  }
  if (i < n_scenes) cb.reach[i] = 0ull;
  if (i < n_scenes * REACH_BINS) cb.hist[i] = 0;
  if (i < 3) cb.counters[i] = 0;
  if (i >= v.n) return;
  v.ccount[i] = 0;
  v.r_num[i] = 0.0;
  v.r_den[i] = 0.0;
  // the step's prediction, which the contact construction neither reads nor
  // changes (it reads q^n and the velocities)
  if (predict) predict_body(v, i);
}

__device__ __forceinline__ int reach_bin(double r) {
  const int b = (int)(__float_as_uint((float)r) >> 21) - REACH_BIN_BASE;
  return b < 0 ? 0 : (b >= REACH_BINS ? REACH_BINS - 1 : b);
}

// upper edge of a reach bin (every reach in bin b is below it, up to float rounding)
__device__ __forceinline__ double reach_bin_edge(int b) {
  return (double)__uint_as_float((unsigned)(b + REACH_BIN_BASE + 1) << 21);
}

// per-scene maximum reach and reach histogram; lanes of a wavefront that share a
// scene (or a scene and bin) combine before one atomic
template <typename T>
__global__ void __launch_bounds__(256) k_contact_reach(View<T> v, ContactBuf cb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int sc = i < v.n ? v.bscene[i] : -1;
  double reach = 0.0;
  if (i < v.n && contact_body(v, i, sc)) {
    T vw[VW];
    load<T, VW>(v.vel + (size_t)VW * i, vw);
    double vd[6] = {(double)vw[0], (double)vw[1], (double)vw[2], (double)vw[3], (double)vw[4], (double)vw[5]};
    double R = (double)v.half[4 * i + 3];
    reach = R + body_pm(v.scenes[sc], vd, R, v.shape[i]);
    cb.breach[i] = reach;
  } else {
    sc = -1;
  }
  const int lane = __lane_id();
  // maximum, one scene at a time
  bool todo = sc >= 0;
  while (__ballot(todo)) {
    const int leader = __ffsll((long long)__ballot(todo)) - 1;
    const int s0 = __shfl(sc, leader);
    const bool mine = todo && sc == s0;
    double r = mine ? reach : 0.0;
    for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o));
    if (lane == leader) atomicMax(cb.reach + s0, (unsigned long long)__double_as_longlong(r));
    todo = todo && !mine;
  }
  // histogram, one (scene, bin) at a time
  const int key = sc >= 0 ? REACH_BINS * sc + reach_bin(reach) : -1;
  todo = key >= 0;
  while (__ballot(todo)) {
    const unsigned long long act = __ballot(todo);
    const int leader = __ffsll((long long)act) - 1;
    const int k0 = __shfl(key, leader);
    const unsigned long long same = __ballot(todo && key == k0);
    if (lane == leader) atomicAdd(cb.hist + k0, __popcll(same));
    todo = todo && key != k0;
  }
}

// cell = 2 cut: cut covers at least 98 % of the scene's bodies (the bin edge
// above the percentile, rounded up by a factor 1 + 1e-6 against float rounding
// of the binning) and never exceeds the largest reach
__global__ void k_contact_cells(SceneDev* scenes, int n_scenes, const unsigned long long* reach,
                                const int* hist) {
  const int sc = blockIdx.x * blockDim.x + threadIdx.x;
  if (sc >= n_scenes) return;
  const double rmax = __longlong_as_double((long long)reach[sc]);
  if (!(rmax > 0.0)) {
    scenes[sc].cell = 1.0;
    return;
  }
  int total = 0;
  for (int b = 0; b < REACH_BINS; ++b) total += hist[REACH_BINS * sc + b];
  const int need = total - total / 50;
  int cum = 0, pb = REACH_BINS - 1;
  for (int b = 0; b < REACH_BINS; ++b) {
    cum += hist[REACH_BINS * sc + b];
    if (cum >= need) {
      pb = b;
      break;
    }
  }
  const double cut = fmin(rmax, reach_bin_edge(pb) * (1.0 + 1e-6));
  scenes[sc].cell = 2.0 * cut;
}

__device__ __forceinline__ unsigned bucket_of(int sc, int cx, int cy, int cz, int tb) {
  unsigned h = (unsigned)cx * 73856093u ^ (unsigned)cy * 19349663u ^ (unsigned)cz * 83492791u ^
               (unsigned)sc * 2654435761u;
  h ^= h >> 13;
  h *= 0x5bd1e995u;
  h ^= h >> 15;
  return h & (unsigned)(tb - 1);
}

__device__ __forceinline__ void cell_of_pos(const double* c, double cell, int* cc) {
  cc[0] = (int)floor(c[0] / cell);
  cc[1] = (int)floor(c[1] / cell);
  cc[2] = (int)floor(c[2] / cell);
}

template <typename T>
__device__ __forceinline__ void centre_of(const View<T>& v, int i, double* c) {
  const T* q = v.qn + (size_t)Rec<T>::Q * i;
  c[0] = pos_value(q, 0);
  c[1] = pos_value(q, 1);
  c[2] = pos_value(q, 2);
}

template <typename T>
__device__ __forceinline__ bool is_large(const View<T>& v, const ContactBuf& cb, int i, int sc) {
  return cb.breach[i] > 0.5 * v.scenes[sc].cell;
}

template <typename T>
__global__ void k_hash_count(View<T> v, ContactBuf cb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.n) return;
  const int sc = v.bscene[i];
  if (!contact_body(v, i, sc)) return;
  if (is_large(v, cb, i, sc)) {
    cb.large[atomicAdd(cb.counters, 1)] = i;
    return;
  }
  double c[3];
  int cc[3];
  centre_of(v, i, c);
  cell_of_pos(c, v.scenes[sc].cell, cc);
  atomicAdd(cb.bucket_count + bucket_of(sc, cc[0], cc[1], cc[2], cb.tb), 1);
}

template <typename T>
__global__ void k_hash_fill(View<T> v, ContactBuf cb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.n) return;
  const int sc = v.bscene[i];
  if (!contact_body(v, i, sc) || is_large(v, cb, i, sc)) return;
  double c[3];
  int cc[3];
  centre_of(v, i, c);
  cell_of_pos(c, v.scenes[sc].cell, cc);
  BroadRec r;
  r.c[0] = (float)c[0];
  r.c[1] = (float)c[1];
  r.c[2] = (float)c[2];
  r.reach = (float)cb.breach[i];
  r.body = i;
  r.scene = sc;
  r.cell = pack_cell(cc[0], cc[1], cc[2]);
  const unsigned b = bucket_of(sc, cc[0], cc[1], cc[2], cb.tb);
  const int pos = atomicAdd(cb.bucket_fill + b, 1);
  cb.rec[cb.bucket_start[b] + pos] = r;
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

// write one bond end into the owner's slot list (stiffness as h^2 kappa_c)
template <typename T>
__device__ __forceinline__ void push_end(const View<T>& v, int owner, int sc, int partner,
                                         int feature, int side, const double* xs,
                                         const double* xo, const double* n, double kap,
                                         double mu) {
  const SceneDev& S = v.scenes[sc];
  const int slot = atomicAdd(v.ccount + owner, 1);
  if (slot >= S.ccap) {
    atomicOr(v.health + sc, 2);
    return;
  }
  const size_t e = ce_base(S, owner) + slot;
  StageRec<T>& r = v.ce_stage[e];
  if constexpr (sizeof(T) == 4) {
    // stiffness and friction coefficient come from the q records and the scene
    double uv[2];
    oct_encode(n, uv);
    const T C[8] = {(T)xs[0], (T)xs[1], (T)xs[2], (T)uv[0], (T)xo[0], (T)xo[1], (T)xo[2], (T)uv[1]};
    store<T, 8>(r.C, C);
  } else {
    const T C[CW] = {(T)xs[0], (T)xs[1], (T)xs[2], (T)kap, (T)xo[0], (T)xo[1], (T)xo[2], (T)mu,
                     (T)n[0], (T)n[1], (T)n[2], (T)0};
    store<T, CW>(r.C, C);
  }
  r.partner = partner;
  r.pad = 0;
  r.key = ((unsigned long long)(unsigned)(partner + 1) << 32) |
          ((unsigned long long)(unsigned)feature << 1) | (unsigned)side;
}

template <typename T>
__device__ __forceinline__ void emit_contact(const View<T>& v, const ContactBuf& cb, int sc,
                                             int i, int j, int feature, const double* xi,
                                             const double* xj, const double* n) {
  const SceneDev& S = v.scenes[sc];
  double m = fmax(free_mass(v, cb, i), free_mass(v, cb, j));
  double kap = S.kscale * m;  // h^2 kappa_c, kappa_c = scale m / h^2
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

// the k-th of three values (k known only at run time) by selects, so that no
// array needs memory to be indexed
__device__ __forceinline__ double pick3(const double* a, int k) {
  return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]);
}

// box-box, vertex-face: reference face = face axis (3 of i, then 3 of j) of least
// overlap; incident vertices within the margin of that face and inside its
// lateral extent become contacts (incident box = i side, reference box = j side).
// All loops are unrolled and run-time choices are selects, so the geometry stays
// in registers.
template <typename T>
__device__ __forceinline__ void narrow_box_box(const View<T>& v, const ContactBuf& cb, int sc, int bi,
                                               int bj, const BodyGeo<T>& gi, const BodyGeo<T>& gj,
                                               double pm) {
  const double dc[3] = {gj.c[0] - gi.c[0], gj.c[1] - gi.c[1], gj.c[2] - gi.c[2]};
  int best = -1;
  double best_ov = 0.0;
  bool apart = false;
#pragma unroll
  for (int ax = 0; ax < 6; ++ax) {
    const double* A = ax < 3 ? gi.A : gj.A;
    const int k = ax % 3;
    const double u[3] = {A[k], A[3 + k], A[6 + k]};
    double ri = 0.0, rj = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      ri += gi.he[m] * fabs(u[0] * gi.A[m] + u[1] * gi.A[3 + m] + u[2] * gi.A[6 + m]);
      rj += gj.he[m] * fabs(u[0] * gj.A[m] + u[1] * gj.A[3 + m] + u[2] * gj.A[6 + m]);
    }
    const double ov = ri + rj - fabs(u[0] * dc[0] + u[1] * dc[1] + u[2] * dc[2]);
    if (ov < -pm) apart = true;
    if (best < 0 || ov < best_ov) {
      best = ax;
      best_ov = ov;
    }
  }
  if (apart) return;
  const bool ref_is_i = best < 3;
  const int k = best % 3;
  double RA[9], IA[9], Rc[3], Ic[3], Rhe[3], Ihe[3];
#pragma unroll
  for (int m = 0; m < 9; ++m) {
    RA[m] = ref_is_i ? gi.A[m] : gj.A[m];
    IA[m] = ref_is_i ? gj.A[m] : gi.A[m];
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    Rc[m] = ref_is_i ? gi.c[m] : gj.c[m];
    Ic[m] = ref_is_i ? gj.c[m] : gi.c[m];
    Rhe[m] = ref_is_i ? gi.he[m] : gj.he[m];
    Ihe[m] = ref_is_i ? gj.he[m] : gi.he[m];
  }
  const int ref = ref_is_i ? bi : bj, inc = ref_is_i ? bj : bi;
  const double ax[3] = {pick3(RA, k), pick3(RA + 3, k), pick3(RA + 6, k)};
  const double tw = ax[0] * (Ic[0] - Rc[0]) + ax[1] * (Ic[1] - Rc[1]) + ax[2] * (Ic[2] - Rc[2]);
  const double sgn = tw >= 0.0 ? 1.0 : -1.0;
  const double nw[3] = {sgn * ax[0], sgn * ax[1], sgn * ax[2]};
  const double hek = pick3(Rhe, k);
#pragma unroll
  for (int vtx = 0; vtx < 8; ++vtx) {
    double xv[3], p[3], rel[3], pl[3];
    vertex_of(vtx, Ihe, xv);
    mat_vec(IA, xv, p);
#pragma unroll
    for (int r = 0; r < 3; ++r) rel[r] = p[r] + Ic[r] - Rc[r];
    mat_tvec(RA, rel, pl);
    const double gap = sgn * pick3(pl, k) - hek;
    if (!(gap < pm) || gap < -2.0 * hek) continue;
    bool lateral = true;
#pragma unroll
    for (int m = 0; m < 3; ++m)
      if (m != k && fabs(pl[m]) > Rhe[m] + pm) lateral = false;
    if (!lateral) continue;
    double xs[3];
#pragma unroll
    for (int m = 0; m < 3; ++m)
      xs[m] = m == k ? sgn * Rhe[m] : (pl[m] < -Rhe[m] ? -Rhe[m] : (pl[m] > Rhe[m] ? Rhe[m] : pl[m]));
    emit_contact(v, cb, sc, inc, ref, vtx, xv, xs, nw);
  }
}

// sphere s (i side) against box b (j side)
template <typename T>
__device__ __forceinline__ void narrow_sphere_box(const View<T>& v, const ContactBuf& cb, int sc, int s,
                                                  int b, const BodyGeo<T>& gs, const BodyGeo<T>& gb,
                                                  double pm) {
  const double r = gs.he[0];
  double rel[3] = {gs.c[0] - gb.c[0], gs.c[1] - gb.c[1], gs.c[2] - gb.c[2]}, pl[3], q[3], nl[3];
  mat_tvec(gb.A, rel, pl);
  bool inside = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    q[k] = pl[k] < -gb.he[k] ? -gb.he[k] : (pl[k] > gb.he[k] ? gb.he[k] : pl[k]);
    if (q[k] != pl[k]) inside = false;
  }
  double gap;
  if (inside) {
    int ks = 0;
    double bestd = gb.he[0] - fabs(pl[0]);
#pragma unroll
    for (int k = 1; k < 3; ++k)
      if (gb.he[k] - fabs(pl[k]) < bestd) {
        bestd = gb.he[k] - fabs(pl[k]);
        ks = k;
      }
    const double sg = pick3(pl, ks) >= 0.0 ? 1.0 : -1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k == ks) q[k] = sg * gb.he[k];
      nl[k] = k == ks ? sg : 0.0;
    }
    gap = -bestd - r;
  } else {
    const double dl[3] = {pl[0] - q[0], pl[1] - q[1], pl[2] - q[2]};
    const double dist = sqrt(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
    if (dist == 0.0) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) nl[k] = dl[k] / dist;
    gap = dist - r;
  }
  if (!(gap < pm)) return;
  double nw[3], pw[3], xi[3];
  mat_vec(gb.A, nl, nw);
#pragma unroll
  for (int k = 0; k < 3; ++k) pw[k] = -r * nw[k];
  mat_tvec(gs.A, pw, xi);
  emit_contact(v, cb, sc, s, b, 8, xi, q, nw);
}

template <typename T>
__device__ __forceinline__ void narrow_pair(const View<T>& v, const ContactBuf& cb, int sc, int i, int j,
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

// ---- broad phase ---------------------------------------------------------------

// Candidate pairs of one workgroup, gathered in LDS (one LDS atomic per pair) and
// appended to the global list with one global atomic per workgroup; a pair that
// does not fit the LDS buffer goes straight to the global list.
constexpr int PAIR_LDS = 4096;  // a workgroup's candidate pairs before one global append

struct PairBuf {
  int2* buf;  // [PAIR_LDS] in LDS
  int* count;
  int* base;
};

__device__ __forceinline__ void global_pair(const ContactBuf& cb, int* health, int sc, int i, int j) {
  const int slot = atomicAdd(cb.counters + 1, 1);
  if (slot < cb.pcap) cb.pairs[slot] = make_int2(i, j);
  else atomicOr(health + sc, 2);
}

__device__ __forceinline__ void append_pair(const PairBuf& pb, const ContactBuf& cb, int* health, int sc,
                                            int i, int j) {
  const int k = atomicAdd(pb.count, 1);
  if (k < PAIR_LDS) pb.buf[k] = make_int2(i, j);
  else global_pair(cb, health, sc, i, j);
}

// every thread of the workgroup calls this once, after its last append
template <typename T>
__device__ __forceinline__ void flush_pairs(const PairBuf& pb, const View<T>& v, const ContactBuf& cb) {
  __syncthreads();
  const int n = min(*pb.count, PAIR_LDS);
  if (threadIdx.x == 0) *pb.base = n > 0 ? atomicAdd(cb.counters + 1, n) : 0;
  __syncthreads();
  const int base = *pb.base;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int2 pr = pb.buf[k];
    if (base + k < cb.pcap) cb.pairs[base + k] = pr;
    else atomicOr(v.health + v.bscene[pr.x], 2);
  }
}

// conservative bounding-sphere test (the narrow phase repeats it exactly)
__device__ __forceinline__ bool spheres_near(const double* a, double ra, const double* b, double rb) {
  const double d0 = b[0] - a[0], d1 = b[1] - a[1], d2 = b[2] - a[2];
  const double r = (ra + rb) * (1.0 + 1e-12);
  return d0 * d0 + d1 * d1 + d2 * d2 < r * r;
}

// the same against a float record: the slack covers float rounding of the
// record's centre (2^-24 relative per coordinate) and reach
__device__ __forceinline__ bool near_rec(const double* a, double ra, const BroadRec& r) {
  const double b0 = r.c[0], b1 = r.c[1], b2 = r.c[2], rb = r.reach;
  const double d0 = b0 - a[0], d1 = b1 - a[1], d2 = b2 - a[2];
  const double mag = fmax(fabs(b0), fmax(fabs(b1), fabs(b2)));
  const double rr = (ra + rb) * (1.0 + 1e-6) + 1e-6 * mag;
  return d0 * d0 + d1 * d1 + d2 * d2 < rr * rr;
}

// pair filters shared by both broad kernels
__device__ __forceinline__ bool pair_allowed(bool pin_i, int group_i, unsigned flags_j, int group_j) {
  if (flags_j & F_NOCONTACT) return false;
  if (pin_i && (flags_j & F_PINNED)) return false;
  if (group_i != 0 && group_j == group_i) return false;
  return true;
}

template <typename T>
__device__ void plane_contacts(const View<T>& v, const ContactBuf& cb, int sc, int i,
                               const BodyGeo<T>& gi, double pmi) {
  const SceneDev& S = v.scenes[sc];
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

template <typename T>
__device__ __forceinline__ double own_pm(const View<T>& v, int i, int sc, const BodyGeo<T>& g) {
  T vw[VW];
  load<T, VW>(v.vel + (size_t)VW * i, vw);
  const double vd[6] = {(double)vw[0], (double)vw[1], (double)vw[2], (double)vw[3], (double)vw[4], (double)vw[5]};
  return body_pm(v.scenes[sc], vd, g.R, g.shape);
}

// BLPB lanes per body: the first lane does the plane contacts; then, for a
// small body, the lanes split the 14 cells made of its own cell (partners of
// higher index) and the 13 cells of the forward half of its neighbourhood, so
// each pair of neighbouring cells is searched from one side only.  One cell per
// lane: each lane's loads form one short dependent chain (bucket range, then
// records), which keeps small scenes from waiting on fourteen such chains in a
// row (1, 2, 7 and 14 lanes were measured; 14 was fastest on every contact
// workload)
constexpr int BLPB = 14;

template <typename T>
__global__ void __launch_bounds__(256) k_broad_small(View<T> v, ContactBuf cb) {
  __shared__ int2 lbuf[PAIR_LDS];
  __shared__ int lcount, lbase;
  if (threadIdx.x == 0) lcount = 0;
  __syncthreads();
  const PairBuf pb{lbuf, &lcount, &lbase};
  const long long gt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(gt / BLPB), sub = (int)(gt % BLPB);
  const int sc = i < v.n ? v.bscene[i] : -1;
  if (i < v.n && contact_body(v, i, sc)) {
    const SceneDev& S = v.scenes[sc];
    const bool pin_i = (v.flags[i] & F_PINNED) != 0;
    if (sub == 0 && !pin_i && S.n_planes > 0) {
      BodyGeo<T> gi;
      body_geo(v, i, gi);
      plane_contacts(v, cb, sc, i, gi, own_pm(v, i, sc, gi));
    }
    if (!is_large(v, cb, i, sc)) {
      double c[3];
      int cc[3];
      centre_of(v, i, c);
      cell_of_pos(c, S.cell, cc);
      const double ri = cb.breach[i];
      const int group_i = v.group[i];
      // the 14 bucket ranges first, so that their loads are in flight together
      constexpr int NC = (14 + BLPB - 1) / BLPB;
      int e0s[NC], e1s[NC];
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        const int t = 13 + sub + u * BLPB;
        e0s[u] = e1s[u] = 0;
        if (t < 27) {
          const unsigned b = bucket_of(sc, cc[0] + t % 3 - 1, cc[1] + (t / 3) % 3 - 1, cc[2] + t / 9 - 1, cb.tb);
          e0s[u] = cb.bucket_start[b];
          e1s[u] = cb.bucket_start[b + 1];
        }
      }
#pragma unroll
      for (int u = 0; u < NC; ++u) {  // offset t: own cell (13), then forward half
        const int t = 13 + sub + u * BLPB;
        const int tx = cc[0] + t % 3 - 1, ty = cc[1] + (t / 3) % 3 - 1, tz = cc[2] + t / 9 - 1;
        const unsigned long long key = pack_cell(tx, ty, tz);
        for (int e = e0s[u]; e < e1s[u]; ++e) {
          const BroadRec r = cb.rec[e];
          if (r.cell != key || r.scene != sc || (t == 13 && r.body <= i)) continue;
          if (!near_rec(c, ri, r)) continue;
          const int j = r.body;
          if (!pair_allowed(pin_i, group_i, v.flags[j], v.group[j])) continue;
          append_pair(pb, cb, v.health, sc, min(i, j), max(i, j));
        }
      }
    }
  }
  flush_pairs(pb, v, cb);
}

// A large body's share of the broad phase, split into tasks of BL_CHUNK
// threads: its cells (those within its reach plus the cut of its centre's
// cell), one per thread, then one pass over the large list for large partners
// of higher index; or, when its cells would outnumber the scene's bodies, the
// scene's bodies, one per thread.  The tasks of all large bodies are spread over
// the grid, so one body with a long reach (a robot's torso over a bed of small
// spheres: tens of thousands of cells) no longer keeps one workgroup busy while
// the others idle.
constexpr int BL_CHUNK = 256;  // threads of k_broad_large

struct LargeWork {
  double c[3], rL, cell;
  int m, w, ncell, tasks;
  bool by_cells;
};

template <typename T>
__device__ __forceinline__ LargeWork large_work(const View<T>& v, const ContactBuf& cb, int L) {
  LargeWork lw;
  const SceneDev& S = v.scenes[v.bscene[L]];
  lw.cell = S.cell;
  const double cut = 0.5 * lw.cell;
  centre_of(v, L, lw.c);
  lw.rL = cb.breach[L];
  // small partners lie within rL + cut of the centre: cells within m of its own
  const double md = ceil((lw.rL + cut) / lw.cell);
  const double span = 2.0 * md + 1.0;
  lw.by_cells = span * span * span <= (double)S.n_bodies;
  lw.m = lw.by_cells ? (int)md : 0;
  lw.w = 2 * lw.m + 1;
  lw.ncell = lw.by_cells ? lw.w * lw.w * lw.w : 0;
  lw.tasks = lw.by_cells ? (lw.ncell + BL_CHUNK - 1) / BL_CHUNK + 1 : (S.n_bodies + BL_CHUNK - 1) / BL_CHUNK;
  return lw;
}

// the first task of every large body (exclusive prefix) and their total; one
// workgroup of 1024 threads
template <typename T>
__global__ void __launch_bounds__(1024) k_large_tasks(View<T> v, ContactBuf cb) {
  __shared__ int part[1024];
  const int nl = cb.counters[0];
  int carry = 0;
  for (int base = 0; base < nl; base += 1024) {
    const int l = base + (int)threadIdx.x;
    const int t = l < nl ? large_work(v, cb, cb.large[l]).tasks : 0;
    part[threadIdx.x] = t;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan
      const int x = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
      __syncthreads();
      part[threadIdx.x] += x;
      __syncthreads();
    }
    if (l < nl) cb.ltask[l] = carry + part[threadIdx.x] - t;
    carry += part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cb.ltask[nl] = carry;
    cb.counters[2] = carry;
  }
}

// grid-stride over the large bodies' tasks
template <typename T>
__global__ void __launch_bounds__(BL_CHUNK) k_broad_large(View<T> v, ContactBuf cb) {
  __shared__ int2 lbuf[PAIR_LDS];
  __shared__ int lcount, lbase;
  if (threadIdx.x == 0) lcount = 0;
  __syncthreads();
  const PairBuf pb{lbuf, &lcount, &lbase};
  const int nl = cb.counters[0], total = cb.counters[2];
  for (int task = blockIdx.x; task < total; task += gridDim.x) {
    // the large body holding this task: the last l with ltask[l] <= task
    int lo = 0, hi = nl - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (cb.ltask[mid] <= task) lo = mid;
      else hi = mid - 1;
    }
    const int L = cb.large[lo];
    const int part = task - cb.ltask[lo];
    const LargeWork lw = large_work(v, cb, L);
    const int sc = v.bscene[L];
    const SceneDev& S = v.scenes[sc];
    const bool pin_L = (v.flags[L] & F_PINNED) != 0;
    const int group_L = v.group[L];
    if (lw.by_cells && part < lw.tasks - 1) {
      const int t = part * BL_CHUNK + (int)threadIdx.x;
      if (t < lw.ncell) {
        const int m = lw.m, w = lw.w;
        int cc[3];
        cell_of_pos(lw.c, lw.cell, cc);
        const int tx = cc[0] + t % w - m, ty = cc[1] + (t / w) % w - m, tz = cc[2] + t / (w * w) - m;
        const unsigned long long key = pack_cell(tx, ty, tz);
        const unsigned b = bucket_of(sc, tx, ty, tz, cb.tb);
        const int e1 = cb.bucket_start[b + 1];
        for (int e = cb.bucket_start[b]; e < e1; ++e) {
          const BroadRec r = cb.rec[e];
          if (r.cell != key || r.scene != sc) continue;
          if (!near_rec(lw.c, lw.rL, r)) continue;
          if (!pair_allowed(pin_L, group_L, v.flags[r.body], v.group[r.body])) continue;
          append_pair(pb, cb, v.health, sc, min(L, r.body), max(L, r.body));
        }
      }
    } else if (lw.by_cells) {
      // large partners of higher index in the same scene
      for (int q = (int)threadIdx.x; q < nl; q += BL_CHUNK) {
        const int j = cb.large[q];
        if (j <= L || v.bscene[j] != sc) continue;
        if (!pair_allowed(pin_L, group_L, v.flags[j], v.group[j])) continue;
        double cj[3];
        centre_of(v, j, cj);
        if (spheres_near(lw.c, lw.rL, cj, cb.breach[j])) append_pair(pb, cb, v.health, sc, L, j);
      }
    } else {
      // the scene's bodies: every small one, and large ones of higher index
      const int j = S.body_off + part * BL_CHUNK + (int)threadIdx.x;
      if (j < S.body_off + S.n_bodies && j != L && contact_body(v, j, sc) &&
          !(is_large(v, cb, j, sc) && j < L) &&
          pair_allowed(pin_L, group_L, v.flags[j], v.group[j])) {
        double cj[3];
        centre_of(v, j, cj);
        if (spheres_near(lw.c, lw.rL, cj, cb.breach[j])) append_pair(pb, cb, v.health, sc, min(L, j), max(L, j));
      }
    }
  }
  flush_pairs(pb, v, cb);
}

// A single scene of few bodies, [first, first + n): every pair tested directly,
// one thread per pair, and one thread per body for its plane contacts.  The
// candidate rule is the broad kernels' (bounding spheres of reach R + pm, the
// same filters), so the pairs proposed are the same; only the spatial hash and
// its eight launches are gone.  The narrow phase repeats the exact test and the
// sort fixes the order, so the contact set and its order do not depend on which
// broad phase found the pairs.
template <typename T>
__global__ void __launch_bounds__(256) k_broad_brute(View<T> v, ContactBuf cb, int first, int n) {
  __shared__ int2 lbuf[PAIR_LDS];
  __shared__ int lcount, lbase;
  if (threadIdx.x == 0) lcount = 0;
  __syncthreads();
  const PairBuf pb{lbuf, &lcount, &lbase};
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long npairs = (long long)n * (n - 1) / 2;
  if (t < n) {
    const int i = first + (int)t;
    const int sc = v.bscene[i];
    if (contact_body(v, i, sc) && !(v.flags[i] & F_PINNED) && v.scenes[sc].n_planes > 0) {
      BodyGeo<T> gi;
      body_geo(v, i, gi);
      plane_contacts(v, cb, sc, i, gi, own_pm(v, i, sc, gi));
    }
  } else if (t < n + npairs) {
    // pair p = b (b - 1) / 2 + a with 0 <= a < b < n
    const long long p = t - n;
    long long b = (long long)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
    while (b * (b - 1) / 2 > p) --b;
    while ((b + 1) * b / 2 <= p) ++b;
    const int i = first + (int)(p - b * (b - 1) / 2), j = first + (int)b;
    const int sc = v.bscene[i];
    if (sc == v.bscene[j] && contact_body(v, i, sc) && contact_body(v, j, sc) &&
        pair_allowed((v.flags[i] & F_PINNED) != 0, v.group[i], v.flags[j], v.group[j])) {
      double ci[3], cj[3];
      centre_of(v, i, ci);
      centre_of(v, j, cj);
      if (spheres_near(ci, cb.breach[i], cj, cb.breach[j])) append_pair(pb, cb, v.health, sc, i, j);
    }
  }
  flush_pairs(pb, v, cb);
}

// one thread per candidate pair (grid-stride)
template <typename T>
__global__ void __launch_bounds__(256) k_narrow_pairs(View<T> v, ContactBuf cb) {
  const int np = min(cb.counters[1], cb.pcap);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
    const int2 pr = cb.pairs[p];
    const int i = pr.x, j = pr.y;
    const int sc = v.bscene[i];
    BodyGeo<T> gi;
    body_geo(v, i, gi);
    narrow_pair(v, cb, sc, i, j, gi, own_pm(v, i, sc, gi));
  }
}

// each body's ends from the staging slots to their final slots in key order
// (keys of one body are distinct: partner, feature, side).  One wave per body:
// lane l holds the keys of slots l, l + 64, ... (up to SORT_REG of them); each
// key is broadcast from its lane in turn and every lane counts the keys below
// its own, which is the slot's rank.  Bodies with more ends than the registers
// hold count against the keys in memory instead.
constexpr int SORT_REG = 4;

__device__ __forceinline__ unsigned long long lane_key(unsigned long long k, int src) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(k & 0xffffffffull), src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(k >> 32), src);
  return ((unsigned long long)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ void move_end(const View<T>& v, size_t base, int from, int to,
                                         unsigned long long key) {
  constexpr int W = ContactRec<T>::W;
  const StageRec<T>& r = v.ce_stage[base + from];
  T C[W];
  load<T, W>(r.C, C);
  store<T, W>(v.ce + W * (base + to), C);
  v.ce_partner[base + to] = r.partner;
  v.ce_key[base + to] = key;
}

template <typename T>
__global__ void __launch_bounds__(64) k_sort_contacts(View<T> v) {
  const int i = blockIdx.x;  // the whole wave works on body i
  if (i >= v.n) return;
  const int sc = v.bscene[i];
  if (!contact_body(v, i, sc)) return;
  const int cap = v.scenes[sc].ccap;
  int cnt = v.ccount[i];
  if (cnt > cap) cnt = cap;
  if (cnt <= 0) return;
  const int lane = threadIdx.x;
  const size_t base = ce_base(v.scenes[sc], i);
  const StageRec<T>* st = v.ce_stage + base;
  if (cnt <= 64 * SORT_REG) {
    const int rounds = (cnt + 63) / 64;
    unsigned long long k[SORT_REG];
    int r[SORT_REG];
#pragma unroll
    for (int u = 0; u < SORT_REG; ++u) {
      const int a = lane + 64 * u;
      k[u] = a < cnt ? st[a].key : ~0ull;
      r[u] = 0;
    }
    for (int b = 0; b < cnt; ++b) {
      const int u = b >> 6;  // wave-uniform
      const unsigned long long own = u == 0 ? k[0] : u == 1 ? k[1] : u == 2 ? k[2] : k[3];
      const unsigned long long kb = lane_key(own, b & 63);
#pragma unroll
      for (int w = 0; w < SORT_REG; ++w)
        if (w < rounds) r[w] += k[w] > kb ? 1 : 0;
    }
#pragma unroll
    for (int u = 0; u < SORT_REG; ++u) {
      const int a = lane + 64 * u;
      if (a < cnt) move_end(v, base, a, r[u], k[u]);
    }
  } else {
    for (int a = lane; a < cnt; a += 64) {
      const unsigned long long key = st[a].key;
      int r = 0;
      for (int b = 0; b < cnt; ++b) r += st[b].key < key ? 1 : 0;
      move_end(v, base, a, r, key);
    }
  }
}

}  // namespace pabd
