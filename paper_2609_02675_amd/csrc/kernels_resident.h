// kernels_resident.h -- whole steps of one scene per workgroup: the prediction,
// the K global/local Jacobi iterations of Algorithm 1 and the velocity recovery
// of a scene that is not tiled (contacts, more bodies than a tile, driven or
// variable bonds) but whose bodies' q^k fit the workgroup's LDS.  The bodies
// exchange q^k through two LDS buffers behind one barrier per iteration, so an
// iteration waits on no global load of a partner's state and a step is one
// launch after its contact construction instead of one launch per iteration.
// Each body's iteration is the flat path's own code (iterate_body) with LDS as
// the source of q^k: a scene gives the same bits here whichever other scenes
// share its batch, and its residual and step counter are kept here.
#pragma once

#include "common.h"
#include "device_math.h"
#include "kernels_flat.h"
#include "kernels_step.h"

namespace pabd {

// workgroup size and the most bodies a resident scene may have (two LDS q
// buffers of RMAX records): 1,024 threads and bodies in FP32 (128 KB), 512 in
// FP64 (96 KB), where the iteration needs more registers per lane
template <typename T>
struct Resident;
template <>
struct Resident<float> {
  static constexpr int NT = 1024, RMAX = 1024;
};
template <>
struct Resident<double> {
  static constexpr int NT = 512, RMAX = 512;
};

// the driven bonds of the scenes in the lists (Sec. 5.3.3, read as in
// k_update_driven) and the FP64 masses the refactor needs: a resident scene
// with driven bonds turns their anchors and refactors its bodies' blocks at
// the start of its step, as the flat path's k_update_driven and k_factor do
struct DrivenTable {
  int n;
  const int *scene, *end_i, *end_j;
  const double *param, *mass64;
};

// list: scene slots, one workgroup each (entries past *n_list leave at once, so
// the grid can stay fixed while scenes come and go); CONTACT: the list holds
// the contact scenes.  LPB lanes per body as in the flat iteration: four for
// contact scenes (their ends split among them), one otherwise; a scene larger
// than NT / LPB bodies takes several passes per iteration.
// ENDS as for iterate_body: 1 when no listed scene has variable ends, 2 otherwise,
// so that each variant carries one loop over the static ends; DRIVEN when the
// scenes have driven bonds (the variants without carry no refactor code)
template <typename T, int LPB, bool CONTACT, int ENDS, bool DRIVEN>
__global__ void __launch_bounds__(Resident<T>::NT) k_resident_step(View<T> v, const int* list, const int* n_list,
                                                                   DrivenTable dt) {
  constexpr int QR = Rec<T>::Q, NT = Resident<T>::NT, RMAX = Resident<T>::RMAX, BPP = NT / LPB;
  __shared__ __align__(16) T lq[2][RMAX * QR];
  __shared__ double rn[NT], rd[NT];
  if ((int)blockIdx.x >= *n_list) return;
  const int sc = list[blockIdx.x];
  const int t = threadIdx.x;
  const SceneDev& S = v.scenes[sc];
  if (S.step >= S.steps_total || S.n_bodies > RMAX) return;
  const int off = S.body_off, n = S.n_bodies, K = S.iters;
  if (DRIVEN && dt.n > 0) {
    // driven anchors at this step's time, then every block of the scene
    // refactored (the same functions as the flat path's kernels)
    bool any = false;
    for (int b = t; b < dt.n; b += NT)
      if (dt.scene[b] == sc) {
        update_driven_entry(v, b, sc, dt.end_i, dt.end_j, dt.param);
        any = true;
      }
    if (__syncthreads_or(any)) {
      for (int b = t; b < n; b += NT) factor_body(v, dt.mass64, off + b);
      __syncthreads();
    }
  }
  // prediction (Algorithm 1), as k_predict: s in global memory, q^0 = s in LDS;
  // a pinned body keeps q^n, in both buffers
  for (int b = t; b < n; b += NT) {
    const int i = off + b;
    T q[QR];
    load<T, QR>(v.qn + (size_t)QR * i, q);
    if (v.flags[i] & F_PINNED) {
      store<T, QR>(lq[0] + QR * b, q);
      store<T, QR>(lq[1] + QR * b, q);
      store<T, QR>(v.s + (size_t)QR * i, q);
      continue;
    }
    const T h = (T)S.h;
    T vw[VW];
    load<T, VW>(v.vel + (size_t)VW * i, vw);
    T s[QR];
#pragma unroll
    for (int c = 0; c < QR; ++c) s[c] = q[c];
    pos_add_lo(s, h * (vw[0] + h * (T)S.g0), h * (vw[1] + h * (T)S.g1), h * (vw[2] + h * (T)S.g2));
    predict_rotation(q + 3, vw + 3, h, s + 3);
    store<T, QR>(v.s + (size_t)QR * i, s);
    store<T, QR>(lq[0] + QR * b, s);
    if (v.flags[i] & F_VARIABLE) {
      // augmented ends, warm start (Sec. 5.2.2), as k_predict
      const T ga = (T)S.al_gamma, ag = (T)(S.al_alpha * S.al_gamma);
      for (int e = v.srow[i]; e < v.srow_end[i]; ++e) {
        T* a = v.al + 4 * (size_t)e;
        if (!(a[3] > (T)0)) continue;
        a[0] = fmax(ga * a[0], a[3]);
        a[1] = ag * a[1];
      }
    }
  }
  __syncthreads();
  // K Jacobi iterations: q^k from one LDS buffer, q^{k+1} into the other
  for (int k = 0; k < K; ++k) {
    const T* src = lq[k & 1];
    T* dst = lq[(k + 1) & 1];
    for (int b0 = 0; b0 < n; b0 += BPP) {
      const int b = b0 + t / LPB;  // the same for the LPB lanes of a body
      if (b < n) iterate_body<T, CONTACT, LPB, true, ENDS>(v, k, nullptr, nullptr, off + b, t % LPB, src, dst, off);
    }
    __syncthreads();
  }
  // velocity recovery and health, as the flat path's last iteration does
  const T* qK = lq[K & 1];
  for (int b = t; b < n; b += NT) {
    const int i = off + b;
    if (v.flags[i] & F_PINNED) {
      v.r_num[i] = 0.0;
      v.r_den[i] = 0.0;
      continue;
    }
    T qf[QR], q0[QR];
    load<T, QR>(qK + QR * b, qf);
    load<T, QR>(v.qn + (size_t)QR * i, q0);
    T vw[VW];
    recover_velocity(qf, q0, (T)(1.0 / S.h), vw);
    bool finite = true;
#pragma unroll
    for (int c = 0; c < QR; ++c) finite = finite && isfinite(qf[c]);
#pragma unroll
    for (int c = 0; c < 6; ++c) finite = finite && isfinite(vw[c]);
    if (!finite) atomicOr(v.health + sc, 1);
    pos_renorm(qf);
    store<T, QR>(v.qn + (size_t)QR * i, qf);
    store<T, VW>(v.vel + (size_t)VW * i, vw);
  }
  __syncthreads();  // every body's residual partials written
  // the scene's FP64 residual in a fixed order: thread t sums bodies t, t + NT,
  // ... in order, then a pairwise tree
  double a = 0.0, d = 0.0;
  for (int b = t; b < n; b += NT) {
    a += v.r_num[off + b];
    d += v.r_den[off + b];
  }
  rn[t] = a;
  rd[t] = d;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (t < w) {
      rn[t] += rn[t + w];
      rd[t] += rd[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    v.rho[sc] = rd[0] > 0.0 ? sqrt(rn[0] / rd[0]) : 0.0;
    v.scenes[sc].step += 1;
  }
}

}  // namespace pabd
