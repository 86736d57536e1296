// kernels_flat.h -- the body iteration of the flat path (Algorithm 1's global
// and local step for one body) and the kernels that run it over a flat range
// of bodies:
//   k_iterate   one global + local iteration for every body (Jacobi: reads only
//               q^k, writes q^{k+1} to the other buffer), increment form:
//               dq = H^{-1} (M (s - q^k) + h^2 sum [w J^T (y_o - y_s) + phi^- J^T n
//                    + J^T f_contact]),  then A <- polar rotation (Sec. 4.2.2)
//   k_iterate_waves  the same over a batch's table of wavefronts (CL lanes per
//               body of a contact scene, one per body of any other scene)
// with the force terms of the variable ends (augmented, polynomial, slider) and
// of the contact ends.  The resident step kernel runs the same body iteration.
#pragma once

#include "common.h"
#include "contact_record.h"
#include "device_math.h"
#include "kernels_step.h"

namespace pabd {

// one augmented end (Sec. 5.2.2) with bond vector d = y_o - y_s at iterate k:
// h^2-scaled force and implicit weight of Psi = 1/2 kappa C^2 + lambda C, C = d - l
// (the multiplier's tension beyond kappa l joins the weight), then the
// multiplier and stiffness updates from C; a = (kappa, lambda, l, kappa_start)
template <typename T>
__device__ __forceinline__ T augmented_end(T* a, const T* d, T h2, T beta, T* f) {
  const T kap = a[0], lam = a[1], l = a[2];
  const T dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  T w = kap, phim = lam - kap * l;
  if (phim > (T)0 && dn > (T)1e-12) {
    w += phim / dn;
    phim = (T)0;
  }
  const T sc = dn > (T)1e-12 ? phim / dn : (T)0;
  f[0] = h2 * (w + sc) * d[0];
  f[1] = h2 * (w + sc) * d[1];
  f[2] = h2 * (w + sc) * d[2];
  const T C = dn - l;
  a[1] = kap * C + lam;
  a[0] = kap + beta * fabs(C);
  return h2 * w;  // implicit weight (h^2-scaled) for the block
}

// one polynomial end, Psi = kappa / p (d - l)^p (p even, at most 12): phi =
// kappa (d - l)^{p-1} = kappa sum_k C(p-1, k) d^k (-l)^{p-1-k}; the terms with
// p-1-k even are >= 0 and form phi^+ (implicit weight phi^+ / d), the others
// phi^- (explicit) -- the split of Sec. 4.2.1; a = (kappa, 0, l, -p)
template <typename T>
__device__ __forceinline__ T polynomial_end(const T* a, const T* d, T h2, T* f) {
  const T kap = a[0], l = a[2];
  const int p = (int)(-a[3]);
  const T dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  T lp[12];  // l^j
  lp[0] = (T)1;
#pragma unroll
  for (int j = 1; j < 12; ++j) lp[j] = lp[j - 1] * l;
  T binom = (T)1, dk1 = (T)1, w = (T)0, phim = (T)0;  // dk1 = d^{k-1}
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    if (k >= p) break;
    if (k > 0) binom = binom * (T)(p - k) / (T)k;
    const int j = p - 1 - k;
    T lj = (T)0;
#pragma unroll
    for (int u = 0; u < 12; ++u)
      if (u == j) lj = lp[u];
    if (j % 2 == 0) {
      if (k >= 1) w += binom * dk1 * lj;
    } else {
      phim -= binom * (k >= 1 ? dk1 * dn : (T)1) * lj;
    }
    if (k >= 1) dk1 *= dn;
  }
  w *= kap;
  phim *= kap;
  const T sc = dn > (T)1e-12 ? phim / dn : (T)0;
  f[0] = h2 * (w + sc) * d[0];
  f[1] = h2 * (w + sc) * d[1];
  f[2] = h2 * (w + sc) * d[2];
  return h2 * w;
}

// one slider end (the point-on-line reading of the slider joint of Sec. 5.1).
// d0 = y_o - y_s is the record's bond vector (point side: from the point to the
// line's anchor on the partner; line side: from the own line anchor to the
// partner's point); g = A u is the line's world direction (u the unit axis in
// the line body's frame, A that body's iterate, or u itself for a world line).
// Sets d to the part of d0 across g -- on either side the vector from this end's
// point to the other, with the line-side point at the foot of the
// perpendicular -- and returns t = d0.g / g.g, the foot's distance along u from
// the line anchor as seen from the line side.
template <typename T>
__device__ __forceinline__ T slider_end(const T* d0, const T* A, const T* u, T* d) {
  T g[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) g[r] = A ? A[3 * r] * u[0] + A[3 * r + 1] * u[1] + A[3 * r + 2] * u[2] : u[r];
  const T t = (d0[0] * g[0] + d0[1] * g[1] + d0[2] * g[2]) / (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
#pragma unroll
  for (int r = 0; r < 3; ++r) d[r] = d0[r] - t * g[r];
  return t;
}

// contact end (reading of the paper's contact bond), d = y_o - y_s: stick force
// kappa d acting only while penetrating along n (n from the partner's surface
// towards the owner), tangential part clamped to mu times the normal part; kap
// is h^2 kappa, so the force comes out scaled by h^2 like the bonds'.
// Returns false when separated (no contribution, no implicit weight).
template <typename T>
__device__ __forceinline__ bool contact_end_force(T kap, T mu, const T* n, const T* d, T* f) {
  const T d0 = d[0], d1 = d[1], d2 = d[2];
  const T n0 = n[0], n1 = n[1], n2 = n[2];
  T dn = n0 * d0 + n1 * d1 + n2 * d2;  // = -gap
  if (!(dn > (T)0)) return false;
  T fn = kap * dn;
  T t0 = kap * (d0 - dn * n0), t1 = kap * (d1 - dn * n1), t2 = kap * (d2 - dn * n2);
  T tn2 = t0 * t0 + t1 * t1 + t2 * t2;
  T lim = mu * fn;
  if (tn2 > lim * lim) {
    T sc = lim * rsqrt_(tn2);
    t0 *= sc;
    t1 *= sc;
    t2 *= sc;
  }
  f[0] = fn * n0 + t0;
  f[1] = fn * n1 + t1;
  f[2] = fn * n2 + t2;
  return true;
}

// residual partials of one body: |q_new - q|_M^2 and |q|_M^2
template <typename T>
__device__ __forceinline__ void residual_terms(const T* m, const T* qo, const T* q, double* num,
                                               double* den) {
  T dd[QW];
  pos_diff(qo, q, dd);
#pragma unroll
  for (int c = 3; c < QW; ++c) dd[c] = qo[c] - q[c];
  const T cc[3] = {(T)pos_value(q, 0), (T)pos_value(q, 1), (T)pos_value(q, 2)};
  *num = m_norm2(m, dd, dd);
  *den = m_norm2(m, cc, q);
}

// sum over the LPB consecutive lanes of a body (xor butterfly: every lane gets
// the same bits, since each partial sum is formed from the same two operands)
template <int LPB, typename U>
__device__ __forceinline__ U lane_sum(U x) {
#pragma unroll
  for (int o = 1; o < LPB; o <<= 1) x += __shfl_xor(x, o);
  return x;
}

// One Jacobi iteration.  LPB consecutive lanes share a body: they split its
// static bond ends and contact ends (lane l takes ends l, l + LPB, ...), sum the
// force terms and the contact change of the FP64 block across the lanes, and the
// first lane solves, projects and stores.
//
// q^k is read from qs and q^{k+1} written to qd, the record of body b at
// (b - qoff) QR: the double-buffered global arrays with qoff = 0 for the flat
// kernels, the scene's LDS buffers with qoff = its first body for the resident
// step.  A body runs in the kernel family that its scene's `resident` flag
// names, so the two never both advance it.
// ENDS chooses the loop over the static ends: 0 per wave at run time (below), 1
// the quadratic loop only (the caller knows the scene has no variable end), 2
// the general loop only.
template <typename T, bool CONTACT, int LPB, bool RESIDENT = false, int ENDS = 0>
__device__ __forceinline__ void iterate_body(const View<T>& v, int k, double* rh_num, double* rh_den,
                                             int i, int sub, const T* qs, T* qd, int qoff) {
  constexpr int QR = Rec<T>::Q;
  const int sc = v.bscene[i];
  if (sc < 0) return;
  if (v.flags[i] & F_PINNED) {
    // a pinned body's residual shares stay zero (it never moves); written in
    // the first iteration, before the step's residual reduction reads them
    if (!RESIDENT && k == 0 && sub == 0) {
      v.r_num[i] = 0.0;
      v.r_den[i] = 0.0;
    }
    return;
  }
  const SceneDev& S = v.scenes[sc];
  if ((S.resident != 0) != RESIDENT) return;
  const int K = S.iters;
  if (k >= K || S.step >= S.steps_total) return;
  T q[QR];
  load<T, QR>(qs + (size_t)QR * (i - qoff), q);
  T rb[QW];
#pragma unroll
  for (int c = 0; c < QW; ++c) rb[c] = (T)0;
  T fac[FW];
  bool refactor = false;
  Block dB{};  // contact and augmented part of H^k - H (this lane's ends)
  const bool var = (v.flags[i] & F_VARIABLE) != 0;
  const int e1 = v.srow_end[i];
  // a wave with a body that has variable ends takes the general loop, any
  // other wave the quadratic loop below (a divergent wave would run both loops
  // one after the other).  Both form every end's terms with the same
  // operations in the same order, so the choice does not change the bits.
  bool general;
  if constexpr (ENDS == 1)
    general = false;
  else if constexpr (ENDS == 2)
    general = true;
  else
    general = wave_any(var);
  if (general) {
    // the general loop (augmented, polynomial and slider ends among others),
    // one end at a time
    for (int e = v.srow[i] + sub; e < e1; e += LPB) {
      const int j = v.se_partner[e];
      T E[EW];
      load<T, EW>(v.se + (size_t)EW * e, E);
      T* a = var ? v.al + 4 * (size_t)e : nullptr;
      const T kind = a ? a[3] : (T)0;
      // a slider end's line anchor sits t0 = E[7] along the axis from the given
      // one (a slider's rest length is 0, so E[7] holds no phi^-): the same line,
      // re-anchored near the point every step so that the bond vector, whose
      // across-axis part is the force, stays short (in FP32 a long one would lose
      // that part to rounding)
      T xs[3] = {E[0], E[1], E[2]}, xo[3] = {E[4], E[5], E[6]};
      if (kind == (T)AL_SLIDER_POINT) {
#pragma unroll
        for (int r = 0; r < 3; ++r) xo[r] = fma(E[7], a[r], xo[r]);
      } else if (kind == (T)AL_SLIDER_LINE) {
#pragma unroll
        for (int r = 0; r < 3; ++r) xs[r] = fma(E[7], a[r], xs[r]);
      }
      T d[3], f[3];
      T qj[QR];
      if (j < 0) {
        bond_vec<T>(q, xs, nullptr, xo, d);
      } else {
        load<T, QR>(qs + (size_t)QR * (j - qoff), qj);
        bond_vec<T>(q, xs, qj, xo, d);
      }
      if (kind == (T)AL_SLIDER_POINT) {
        // fixed weight at the own point (in the static block), drawn to the foot
        T dp[3];
        const T t = slider_end(d, j < 0 ? (const T*)nullptr : qj + 3, a, dp);
        end_force(E[3], (T)0, dp, f);
        add_JT(rb, E, f[0], f[1], f[2]);
        if (k == K - 1) v.se[(size_t)EW * e + 7] = E[7] - t;  // the foot is -t from the anchor
      } else if (kind == (T)AL_SLIDER_LINE) {
        // the own point is the foot xf = x_s + t u, so its weight moves every iteration
        T dp[3];
        const T t = slider_end(d, q + 3, a, dp);
        const T xf[3] = {fma(t, a[0], xs[0]), fma(t, a[1], xs[1]), fma(t, a[2], xs[2])};
        end_force(E[3], (T)0, dp, f);
        add_JT(rb, xf, f[0], f[1], f[2]);
        block_add_end(dB, (double)E[3], (double)xf[0], (double)xf[1], (double)xf[2]);
        refactor = true;
        if (k == K - 1) v.se[(size_t)EW * e + 7] = E[7] + t;
      } else if (kind != (T)0) {
        const T w = kind > (T)0 ? augmented_end(a, d, (T)(S.h * S.h), (T)S.al_beta, f)
                                : polynomial_end(a, d, (T)(S.h * S.h), f);
        block_add_end(dB, (double)w, (double)E[0], (double)E[1], (double)E[2]);
        refactor = true;
        add_JT(rb, E, f[0], f[1], f[2]);
      } else {
        quad_end_force(E, d, f);
        add_JT(rb, E, f[0], f[1], f[2]);
      }
    }
  } else {
    // quadratic ends only: the lanes of a body take its ends in turn, two ends
    // per round with both ends' loads (record and partner state) in flight
    // together; each end's terms are still added in end order
    for (int e = v.srow[i] + sub; e < e1; e += 2 * LPB) {
      const int eb = e + LPB;
      const bool hb = eb < e1;
      const int ja = v.se_partner[e];
      const int jb = hb ? v.se_partner[eb] : -1;
      T Ea[EW], Eb[EW], qa[QR], qb[QR];
      load<T, EW>(v.se + (size_t)EW * e, Ea);
      if (hb) load<T, EW>(v.se + (size_t)EW * eb, Eb);
      if (ja >= 0) load<T, QR>(qs + (size_t)QR * (ja - qoff), qa);
      if (jb >= 0) load<T, QR>(qs + (size_t)QR * (jb - qoff), qb);
      T d[3], f[3];
      bond_vec<T>(q, Ea, ja < 0 ? (const T*)nullptr : qa, Ea + 4, d);
      quad_end_force(Ea, d, f);
      add_JT(rb, Ea, f[0], f[1], f[2]);
      if (hb) {
        bond_vec<T>(q, Eb, jb < 0 ? (const T*)nullptr : qb, Eb + 4, d);
        quad_end_force(Eb, d, f);
        add_JT(rb, Eb, f[0], f[1], f[2]);
      }
    }
  }
  if constexpr (CONTACT) {
    int cnt = v.ccount[i];
    if (cnt > S.ccap) cnt = S.ccap;
    const size_t base = ce_base(S, i);
    // the lanes of a body take its ends in turn (neighbouring lanes read
    // neighbouring records), two ends per round with both ends' loads (record
    // and partner state) in flight together
    constexpr int W = ContactRec<T>::W;
    const T mu = (T)S.mu;
    auto contact_end = [&](const T* C, int j, const T* qj) {
      T d[3], f[3], n[3], kap;
      bond_vec<T>(q, C, j < 0 ? nullptr : qj, C + 4, d);
      if constexpr (sizeof(T) == 4) {
        // h^2 kappa from the two q records, the normal from its octahedral form
        kap = fmax(q[Q_KAPPA], j < 0 ? (T)0 : qj[Q_KAPPA]);
        oct_decode(C[3], C[7], n);
      } else {
        kap = C[3];
        n[0] = C[8];
        n[1] = C[9];
        n[2] = C[10];
      }
      if (!contact_end_force(kap, mu, n, d, f)) return;
      add_JT(rb, C, f[0], f[1], f[2]);
      block_add_end(dB, (double)kap, (double)C[0], (double)C[1], (double)C[2]);
      refactor = true;
    };
    // In the flat kernels the next round's partner ids are loaded during this
    // round, so that a round's records and partner states all go out at once
    // instead of the states waiting for the ids.  The resident kernel, whose
    // partner states come from LDS, loads each round's ids at its start (it has
    // no registers to spare for the ids ahead).
    int ja = -1, jb = -1;
    if constexpr (!RESIDENT) {
      if (sub < cnt) {
        ja = v.ce_partner[base + sub];
        jb = sub + LPB < cnt ? v.ce_partner[base + sub + LPB] : -1;
      }
    }
    for (int c = sub; c < cnt; c += 2 * LPB) {
      const int cb = c + LPB;
      const bool hb = cb < cnt;
      if constexpr (RESIDENT) {
        ja = v.ce_partner[base + c];
        jb = hb ? v.ce_partner[base + cb] : -1;
      }
      T Ca[W], Cb[W], qa[QR], qb[QR];
      load<T, W>(v.ce + (size_t)W * (base + c), Ca);
      if (hb) load<T, W>(v.ce + (size_t)W * (base + cb), Cb);
      if (ja >= 0) load<T, QR>(qs + (size_t)QR * (ja - qoff), qa);
      if (jb >= 0) load<T, QR>(qs + (size_t)QR * (jb - qoff), qb);
      int jan = -1, jbn = -1;
      if constexpr (!RESIDENT) {
        const int cn = c + 2 * LPB;
        jan = cn < cnt ? v.ce_partner[base + cn] : -1;
        jbn = cn + LPB < cnt ? v.ce_partner[base + cn + LPB] : -1;
      }
      contact_end(Ca, ja, qa);
      if (hb) contact_end(Cb, jb, qb);
      if constexpr (!RESIDENT) {
        ja = jan;
        jb = jbn;
      }
    }
  }
  if constexpr (LPB > 1) {
#pragma unroll
    for (int c = 0; c < QW; ++c) rb[c] = lane_sum<LPB>(rb[c]);
    {
      refactor = lane_sum<LPB>(refactor ? 1 : 0) > 0;
      if (refactor) {  // uniform across the body's lanes
        dB.a = lane_sum<LPB>(dB.a);
        dB.b0 = lane_sum<LPB>(dB.b0);
        dB.b1 = lane_sum<LPB>(dB.b1);
        dB.b2 = lane_sum<LPB>(dB.b2);
        dB.d00 = lane_sum<LPB>(dB.d00);
        dB.d01 = lane_sum<LPB>(dB.d01);
        dB.d02 = lane_sum<LPB>(dB.d02);
        dB.d11 = lane_sum<LPB>(dB.d11);
        dB.d12 = lane_sum<LPB>(dB.d12);
        dB.d22 = lane_sum<LPB>(dB.d22);
      }
    }
    if (sub != 0) return;
  }
  if (refactor) {  // H^k changed: a contact penetrates, or a variable end's weight or point moved
    const double* bb = v.blk + 10 * (size_t)i;
    const Block B{bb[0] + dB.a,   bb[1] + dB.b0,  bb[2] + dB.b1,  bb[3] + dB.b2,  bb[4] + dB.d00,
                  bb[5] + dB.d01, bb[6] + dB.d02, bb[7] + dB.d11, bb[8] + dB.d12, bb[9] + dB.d22};
    double f64[10];
    block_inverse(B, f64);
#pragma unroll
    for (int c = 0; c < 10; ++c) fac[c] = (T)f64[c];
  } else {
    load<T, FW>(v.fac + (size_t)FW * i, fac);
  }
  T s[QR], m[MW];
  load<T, QR>(v.s + (size_t)QR * i, s);
  load<T, MW>(v.mass + (size_t)MW * i, m);
  T r[QW];  // M (s - q^k) + h^2 sum (...): the forces are already scaled by h^2
#pragma unroll
  for (int c = 0; c < QW; ++c) r[c] = rb[c];
  add_inertia(r, m, s, q);
  T dq[QW];
  block_apply(fac, r, dq);
  T qo[QR];
#pragma unroll
  for (int c = 0; c < QR; ++c) qo[c] = q[c];
  pos_add_lo(qo, dq[0], dq[1], dq[2]);
  T Ah[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) Ah[c] = q[3 + c] + dq[3 + c];
  if (S.debug & 1) {
#pragma unroll
    for (int c = 0; c < 9; ++c) qo[3 + c] = Ah[c];
  } else {
    polar_rotation(Ah, qo + 3, v.polar, i);
  }
  // q^{k+1} for the partners' next iteration; after the flat path's last
  // iteration nothing reads it (the body's step ends below)
  if (RESIDENT || k < K - 1) store<T, QR>(qd + (size_t)QR * (i - qoff), qo);
  if (k == K - 1 || rh_num) {
    double num, den;
    residual_terms(m, qo, q, &num, &den);
    if (k == K - 1) {
      v.r_num[i] = num;
      v.r_den[i] = den;
    }
    if (rh_num) {
      rh_num[(size_t)k * v.n + i] = num;
      rh_den[(size_t)k * v.n + i] = den;
    }
  }
  if constexpr (!RESIDENT) {
    if (k == K - 1) {
      // the end of the body's step on the flat path: velocity recovery (Sec. 4.4)
      // from q^K and q^n, the health bit, and q^{n+1} = q^K with its position
      // folded back to (hi, lo) (the resident kernel ends its scenes' steps itself)
      T q0[QR], vw[VW];
      load<T, QR>(v.qn + (size_t)QR * i, q0);
      // q^K as a value of its own, as if read back from memory: the recovery's
      // subtractions must not fuse with the local step's last products, so
      // that the flat path rounds as the resident kernel does
#pragma unroll
      for (int c = 0; c < QR; ++c) asm volatile("" : "+v"(qo[c]));
      recover_velocity(qo, q0, (T)(1.0 / S.h), vw);
      bool finite = true;
#pragma unroll
      for (int c = 0; c < QR; ++c) finite = finite && isfinite(qo[c]);
#pragma unroll
      for (int c = 0; c < 6; ++c) finite = finite && isfinite(vw[c]);
      if (!finite) atomicOr(v.health + sc, 1);
      pos_renorm(qo);
      store<T, QR>(v.qn + (size_t)QR * i, qo);
      store<T, VW>(v.vel + (size_t)VW * i, vw);
    }
  }
}

// occupancy: at least four waves per SIMD in FP32 (at most 128 registers), two
// in FP64; the iteration waits on loads of its partners and contact records,
// so resident waves matter more than the few registers of its rare paths
template <typename T, bool CONTACT, int LPB>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 4 : 2) k_iterate(View<T> v, int k, double* rh_num, double* rh_den) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / LPB), sub = (int)(t % LPB);
  if (i >= v.n) return;
  iterate_body<T, CONTACT, LPB>(v, k, rh_num, rh_den, i, sub, v.q[k & 1], v.q[(k + 1) & 1], 0);
}

// The same iteration over a table of wavefronts (first body, bodies, lanes per
// body): a wave covers 64 / CL bodies of a contact scene with CL lanes each (16
// with the default four), or 64 bodies of a contact-free scene with one lane
// each, and never spans two scenes.  Waves past the table's count leave at
// once, so the grid can stay fixed while scenes come and go.
struct FlatWave {
  int first, count, lpb, contact;  // lpb: lanes per body (CL for a contact wave, else 1)
};

template <typename T, int CL>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 4 : 2) k_iterate_waves(View<T> v, int k, const FlatWave* waves,
                                                       const int* n_waves) {
  const int w = (int)((blockIdx.x * (long long)blockDim.x + threadIdx.x) / 64);
  const int l = (int)(threadIdx.x & 63);
  if (w >= *n_waves) return;
  const FlatWave fw = waves[w];
  if (fw.contact) {
    if (l / CL >= fw.count) return;
    iterate_body<T, true, CL>(v, k, nullptr, nullptr, fw.first + l / CL, l % CL, v.q[k & 1], v.q[(k + 1) & 1], 0);
  } else {
    if (l >= fw.count) return;
    iterate_body<T, false, 1>(v, k, nullptr, nullptr, fw.first + l, 0, v.q[k & 1], v.q[(k + 1) & 1], 0);
  }
}

}  // namespace pabd
