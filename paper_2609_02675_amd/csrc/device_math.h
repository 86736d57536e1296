// device_math.h -- per-body math of the PABD hot path, templated on the
// arithmetic type (float for the FP32 path, double for the FP64 path).
//
// q = (c, a1, a2, a3) in R^12 with A = [a1, a2, a3]^T (rows), y = A x + c (Sec. 3).
// The 12x12 block H = [[a I, e_k b^T], [b e_k^T, D]] (Sec. 4.3) is kept as the
// FP64 scalars (a, b, D) and its inverse as (alpha, g, G) with
//   b~ = b/a, D~ = D - b b^T / a, G = D~^{-1}, g = G b~, alpha = 1/a + b~^T g,
// so that H^{-1} r = (dc, da_k) with
//   dc_k = alpha r_c[k] - g . r_a[k],   da_k = -g r_c[k] + G r_a[k].
#pragma once

#include <hip/hip_runtime.h>

namespace pabd {

template <typename T>
struct Eps;
// polar_tol2: squared Newton step below which the measured continuation of the
// polar iteration ends (the error left is below polar_tol2 / 2); polar_e_one /
// polar_e_two: det X_1 - 1 after the first step up to which one / two further
// steps leave that same error (sqrt(tol) and (4 tol)^(1/4), rounded down for the
// rounding of the determinant)
template <>
struct Eps<float> {
  static constexpr float polar_tol2 = 1e-7f;
  static constexpr float det_floor = 1e-6f;
  static constexpr float polar_e_one = 3.1e-4f;
  static constexpr float polar_e_two = 2.5e-2f;
};
template <>
struct Eps<double> {
  static constexpr double polar_tol2 = 1e-16;
  static constexpr double det_floor = 1e-12;
  static constexpr double polar_e_one = 0.99e-8;
  static constexpr double polar_e_two = 1.4e-4;
};

template <typename T>
__device__ __forceinline__ T dsqrt(T x) {
  return sqrt(x);
}

// 1/x and 1/sqrt(x): the hardware approximations (about 1 ulp) in FP32, exact
// IEEE operations in FP64
template <typename T>
__device__ __forceinline__ T rcp(T x) {
  if constexpr (sizeof(T) == 4)
    return __builtin_amdgcn_rcpf(x);
  else
    return (T)1 / x;
}
template <typename T>
__device__ __forceinline__ T rsqrt_(T x) {
  if constexpr (sizeof(T) == 4)
    return __builtin_amdgcn_rsqf(x);
  else
    return (T)1 / sqrt(x);
}

// ---- 3x3 helpers (row-major) ------------------------------------------------

template <typename T>
__device__ __forceinline__ void mat_vec(const T* M, const T* x, T* y) {
  y[0] = M[0] * x[0] + M[1] * x[1] + M[2] * x[2];
  y[1] = M[3] * x[0] + M[4] * x[1] + M[5] * x[2];
  y[2] = M[6] * x[0] + M[7] * x[1] + M[8] * x[2];
}

template <typename T>
__device__ __forceinline__ void mat_tvec(const T* M, const T* x, T* y) {
  y[0] = M[0] * x[0] + M[3] * x[1] + M[6] * x[2];
  y[1] = M[1] * x[0] + M[4] * x[1] + M[7] * x[2];
  y[2] = M[2] * x[0] + M[5] * x[1] + M[8] * x[2];
}

// C = cofactor matrix of X (X^{-T} = C / det X); returns det X
template <typename T>
__device__ __forceinline__ T cofactor(const T* X, T* C) {
  C[0] = X[4] * X[8] - X[5] * X[7];
  C[1] = X[5] * X[6] - X[3] * X[8];
  C[2] = X[3] * X[7] - X[4] * X[6];
  C[3] = X[2] * X[7] - X[1] * X[8];
  C[4] = X[0] * X[8] - X[2] * X[6];
  C[5] = X[1] * X[6] - X[0] * X[7];
  C[6] = X[1] * X[5] - X[2] * X[4];
  C[7] = X[2] * X[3] - X[0] * X[5];
  C[8] = X[0] * X[4] - X[1] * X[3];
  return X[0] * C[0] + X[1] * C[1] + X[2] * C[2];
}

// ---- nearest rotation ---------------------------------------------------------

// Cyclic Jacobi on a symmetric 3x3 S (packed s00 s01 s02 s11 s12 s22): eigenvalues
// lam and eigenvectors as columns of V.
template <typename T>
__device__ void sym_eig3(const T* S, T* lam, T* V) {
  T a[3][3] = {{S[0], S[1], S[2]}, {S[1], S[3], S[4]}, {S[2], S[4], S[5]}};
  T v[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int sweep = 0; sweep < 32; ++sweep) {
    T off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    T scale = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (!(off > scale * (T)1e-30)) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      T apq = a[p][q];
      if (apq == (T)0) continue;
      T tau = (a[q][q] - a[p][p]) / ((T)2 * apq);
      T t = (tau >= (T)0 ? (T)1 : (T)-1) / (fabs(tau) + dsqrt(tau * tau + (T)1));
      T c = (T)1 / dsqrt(t * t + (T)1), s = t * c;
      for (int k = 0; k < 3; ++k) {
        T akp = a[k][p], akq = a[k][q];
        a[k][p] = c * akp - s * akq;
        a[k][q] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {
        T apk = a[p][k], aqk = a[q][k];
        a[p][k] = c * apk - s * aqk;
        a[q][k] = s * apk + c * aqk;
      }
      for (int k = 0; k < 3; ++k) {
        T vkp = v[k][p], vkq = v[k][q];
        v[k][p] = c * vkp - s * vkq;
        v[k][q] = s * vkp + c * vkq;
      }
    }
  }
  for (int k = 0; k < 3; ++k) {
    lam[k] = a[k][k];
    for (int r = 0; r < 3; ++r) V[3 * r + k] = v[r][k];
  }
}

// Nearest proper rotation through the two largest singular pairs of A:
// R = u1 v1^T + u2 v2^T + (u1 x u2)(v1 x v2)^T.  Used when Newton cannot run
// (det A <= 0 or nearly singular) or does not converge.
template <typename T>
__device__ void nearest_rotation_svd(const T* A, T* R) {
  T S[6];
  S[0] = A[0] * A[0] + A[3] * A[3] + A[6] * A[6];
  S[1] = A[0] * A[1] + A[3] * A[4] + A[6] * A[7];
  S[2] = A[0] * A[2] + A[3] * A[5] + A[6] * A[8];
  S[3] = A[1] * A[1] + A[4] * A[4] + A[7] * A[7];
  S[4] = A[1] * A[2] + A[4] * A[5] + A[7] * A[8];
  S[5] = A[2] * A[2] + A[5] * A[5] + A[8] * A[8];
  T lam[3], V[9];
  sym_eig3(S, lam, V);
  int i1 = 0;
  for (int k = 1; k < 3; ++k)
    if (lam[k] > lam[i1]) i1 = k;
  int i2 = i1 == 0 ? 1 : 0;
  for (int k = 0; k < 3; ++k)
    if (k != i1 && lam[k] > lam[i2]) i2 = k;
  T v1[3] = {V[i1], V[3 + i1], V[6 + i1]}, v2[3] = {V[i2], V[3 + i2], V[6 + i2]};
  T u1[3], u2[3];
  mat_vec(A, v1, u1);
  mat_vec(A, v2, u2);
  T n1 = dsqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
  if (!(n1 > (T)0)) {  // A == 0: keep identity
    for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? (T)1 : (T)0;
    return;
  }
  for (int k = 0; k < 3; ++k) u1[k] /= n1;
  // u2 orthogonal to u1 (Gram-Schmidt guards rank-one A)
  T d12 = u1[0] * u2[0] + u1[1] * u2[1] + u1[2] * u2[2];
  for (int k = 0; k < 3; ++k) u2[k] -= d12 * u1[k];
  T n2 = dsqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  if (!(n2 > (T)1e-30)) {
    T e[3] = {fabs(u1[0]) < (T)0.6 ? (T)1 : (T)0, fabs(u1[0]) < (T)0.6 ? (T)0 : (T)1, 0};
    T de = u1[0] * e[0] + u1[1] * e[1];
    for (int k = 0; k < 3; ++k) u2[k] = e[k] - de * u1[k];
    n2 = dsqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  }
  for (int k = 0; k < 3; ++k) u2[k] /= n2;
  T u3[3] = {u1[1] * u2[2] - u1[2] * u2[1], u1[2] * u2[0] - u1[0] * u2[2],
             u1[0] * u2[1] - u1[1] * u2[0]};
  T v3[3] = {v1[1] * v2[2] - v1[2] * v2[1], v1[2] * v2[0] - v1[0] * v2[2],
             v1[0] * v2[1] - v1[1] * v2[0]};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) R[3 * r + c] = u1[r] * v1[c] + u2[r] * v2[c] + u3[r] * v3[c];
}

// One Newton step X <- (zeta X + X^{-T} / zeta) / 2 for the orthogonal polar
// factor, in place as X += D with D = (zeta / 2 - 1) X + C / (2 zeta det) (C the
// cofactor matrix, X^{-T} = C / det), and *step2 = |D|^2.  The determinant
// scaling zeta = det^{-1/3} applies only far from orthogonal (near SO(3),
// det ~ 1); *unscaled tells whether the step ran with zeta = 1.  Returns false
// when det X is not safely positive.
template <typename T>
__device__ __forceinline__ bool polar_newton_step(T* X, T* step2, bool* unscaled) {
  T C[9];
  const T det = cofactor(X, C);
  if (!(det > Eps<T>::det_floor)) return false;
  *unscaled = det > (T)0.5 && det < (T)1.5;
  const T zeta = *unscaled ? (T)1 : rcp(cbrt(det));
  const T a = (T)0.5 * zeta - (T)1, b = (T)0.5 * rcp(zeta * det);
  T diff = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const T dk = a * X[k] + b * C[k];
    X[k] += dk;
    diff += dk * dk;
  }
  *step2 = diff;
  return true;
}

// The fast steps work on X = sigma Y with a per-lane scalar sigma: from
// C(X) = sigma^2 C(Y) and det X = sigma^3 det Y, the step
// X' = (zeta X + X^{-T} / zeta) / 2 is sigma' = zeta sigma / 2 with
// Y' = Y + gamma C(Y), gamma = 1 / (zeta^2 sigma^2 det Y): one fma per entry.
//
// An unscaled step (zeta = 1) whose size is not measured, for the lanes with
// on set (only right after a step, when det X >= 1); the other lanes keep Y and
// sigma.  Run by the whole wave, so that no lane's registers need merging
// afterwards.
template <typename T>
__device__ __forceinline__ void polar_newton_plain(T* Y, T* sigma, bool on) {
  T C[9];
  const T det = cofactor(Y, C);
  const T s = *sigma;
  const T g = on ? rcp(s * s * det) : (T)0;
  *sigma = on ? (T)0.5 * s : s;
#pragma unroll
  for (int k = 0; k < 9; ++k) Y[k] = fma(g, C[k], Y[k]);
}

__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }
__device__ __forceinline__ bool wave_all(bool p) { return __builtin_amdgcn_ballot_w64(!p) == 0; }

// Rotation factor of the polar decomposition (local step, Sec. 4.2.2), in place:
// X <- R where X = R S.  Newton's iteration acts on each singular value alone,
// s <- (s + 1/s) / 2 (or (zeta s + 1/(zeta s)) / 2 with a scaling zeta), which
// is at least 1: after the first step every singular value is s_i = 1 + e_i
// with e_i >= 0, so e = det X_1 - 1 = prod (1 + e_i) - 1 >= sum e_i bounds the
// Frobenius error |X_1 - R|.  A further step leaves e_i^2 / (2 (1 + e_i)) per
// singular value, so at most e^2 / 2 in all, and a third e^4 / 8.  The first
// step is not measured; the second takes det X_1 from the cofactors it needs
// anyway, and with the error target tau / 2 (tau = polar_tol2) it ends the
// iteration when e <= polar_e_one (e^2 / 2 < tau / 2), adds a third step when
// e <= polar_e_two (e^4 / 8 < tau / 2), and otherwise hands the lane to the
// measured continuation.  Every Newton iterate has the input's orthogonal
// factor, so if det X is not safely positive or Newton stalls, the nearest
// proper rotation from the SVD of the current iterate is the answer.
template <typename T>
__device__ __forceinline__ bool polar_fast(T* X, bool* ok_out) {
  // first step, not measured: Y = X + g C(X) and sigma = zeta / 2, so that the
  // Newton iterate is X_1 = sigma Y
  T C[9];
  const T det = cofactor(X, C);
  const bool ok = det > Eps<T>::det_floor;
  const bool unscaled = det > (T)0.5 && det < (T)1.5;
  const T zeta = unscaled || !ok ? (T)1 : rcp(cbrt(det));
  const T g = ok ? rcp(zeta * zeta * det) : (T)0;
  T sigma = ok ? (T)0.5 * zeta : (T)1;
#pragma unroll
  for (int k = 0; k < 9; ++k) X[k] = fma(g, C[k], X[k]);
  // second step, measured by the determinant: a Newton step maps every singular
  // value s to (s + 1/s) / 2 >= 1, so e = det X_1 - 1 >= sum (s_i - 1) bounds
  // |X_1 - R|_F, the second step leaves at most e^2 / 2 and a third e^4 / 8
  T C1[9];
  const T det1 = cofactor(X, C1);
  const T e = fma(sigma * sigma * sigma, det1, (T)-1);
  const bool one = ok && unscaled && e <= Eps<T>::polar_e_one;
  const bool two = ok && unscaled && !one && e <= Eps<T>::polar_e_two;
  const T g1 = one || two ? rcp(sigma * sigma * det1) : (T)0;
  sigma = one || two ? (T)0.5 * sigma : sigma;
#pragma unroll
  for (int k = 0; k < 9; ++k) X[k] = fma(g1, C1[k], X[k]);
  if (wave_any(two)) polar_newton_plain<T>(X, &sigma, two);
#pragma unroll
  for (int k = 0; k < 9; ++k) X[k] *= sigma;
  *ok_out = ok;
  return one || two;
}

// The rest for a lane whose first step was too large: measured steps while det X
// stays safely positive, then, if they did not converge, the SVD.  Returns how
// the rotation was found: bit0 = from the SVD (det X not safely positive, or
// Newton stalled), bit1 = det X <= 0 (X is still the input when the first step
// could not run, and Newton iterates keep the sign of the determinant).
template <typename T>
__device__ __forceinline__ int polar_finish(T* X, bool ok) {
  bool done = false;
  int how = 0;
  if (ok) {
    T d2;
    bool unscaled;
#pragma unroll 1
    for (int it = 1; it < 16; ++it) {
      if (!polar_newton_step<T>(X, &d2, &unscaled)) break;
      if (d2 < Eps<T>::polar_tol2) {
        done = true;
        break;
      }
    }
  } else {
    T C[9];
    if (!(cofactor(X, C) > (T)0)) how = 2;
  }
  if (!done) {
    T Y[9];
    nearest_rotation_svd(X, Y);
#pragma unroll
    for (int k = 0; k < 9; ++k) X[k] = Y[k];
    how |= 1;
  }
  return how;
}

// per-body counts of the local step's fallback, 2 per body from `counts`:
// [0] rotations from the SVD, [1] those whose input had det <= 0.  Each body
// is advanced by one lane, which owns its counters, so no atomics; the address
// is formed here, in the rare path, so that callers keep no pointer live
// through the common one.
__device__ __forceinline__ void count_polar(unsigned* counts, int body, int how) {
  if (!counts || !how) return;
  unsigned* cnt = counts + 2 * (size_t)body;
  cnt[0] += (unsigned)(how & 1);
  cnt[1] += (unsigned)((how >> 1) & 1);
}

template <typename T>
__device__ __forceinline__ void polar_rotation_inplace(T* X, unsigned* counts, int body) {
  bool ok;
  const bool done = polar_fast(X, &ok);
  if (wave_any(!done))
    if (!done) count_polar(counts, body, polar_finish(X, ok));
}

// The same for a caller short of registers: around the rare continuation X
// goes through the lane's own 9 words `spill` of LDS, so that the compiler need
// not keep a second copy of X in registers beside the continuation's own.
template <typename T>
__device__ __forceinline__ void polar_rotation_spill(T* X, T* spill, unsigned* counts, int body) {
  bool ok;
  const bool done = polar_fast(X, &ok);
  // spill word w holds X[(w + 1) % 9]: X[1..8] in two 16-byte groups, which
  // for X = q + 3 are register quads of the record q
  if (wave_any(!done)) {
#pragma unroll
    for (int k = 0; k < 9; ++k) spill[(k + 8) % 9] = X[k];
    asm volatile("" ::: "memory");
    if (!done) {
      T Y[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) Y[k] = spill[(k + 8) % 9];
      count_polar(counts, body, polar_finish(Y, ok));
#pragma unroll
      for (int k = 0; k < 9; ++k) spill[(k + 8) % 9] = Y[k];
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int k = 0; k < 9; ++k) X[k] = spill[(k + 8) % 9];
  }
}

template <typename T>
__device__ __forceinline__ void polar_rotation(const T* A, T* R, unsigned* counts, int body) {
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = A[k];
  polar_rotation_inplace(R, counts, body);
}

// ---- prediction (Algorithm 1, prediction loop) ---------------------------------

// A* = R(dQ) A with dQ = normalise(h w / 2, 1) (scalar last): the normalised
// quaternion update Q* = Q + h/2 [w, 0] Q expressed on the rotation matrix.
template <typename T>
__device__ __forceinline__ void predict_rotation(const T* A, const T* w, T h, T* As) {
  T x = (T)0.5 * h * w[0], y = (T)0.5 * h * w[1], z = (T)0.5 * h * w[2];
  T inv = rcp((T)1 + x * x + y * y + z * z);
  T R[9];
  R[0] = (T)1 - (T)2 * (y * y + z * z) * inv;
  R[1] = (T)2 * (x * y - z) * inv;
  R[2] = (T)2 * (x * z + y) * inv;
  R[3] = (T)2 * (x * y + z) * inv;
  R[4] = (T)1 - (T)2 * (x * x + z * z) * inv;
  R[5] = (T)2 * (y * z - x) * inv;
  R[6] = (T)2 * (x * z - y) * inv;
  R[7] = (T)2 * (y * z + x) * inv;
  R[8] = (T)1 - (T)2 * (x * x + y * y) * inv;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      As[3 * r + c] = R[3 * r] * A[c] + R[3 * r + 1] * A[3 + c] + R[3 * r + 2] * A[6 + c];
}

// ---- the 12x12 block (Sec. 4.3) ------------------------------------------------

// FP64 block scalars: a, b[3], D (sym: D00 D01 D02 D11 D12 D22)
struct Block {
  double a, b0, b1, b2, d00, d01, d02, d11, d12, d22;
};

__device__ __forceinline__ void block_add_end(Block& B, double w, double x0, double x1,
                                              double x2) {
  B.a += w;
  B.b0 += w * x0;
  B.b1 += w * x1;
  B.b2 += w * x2;
  B.d00 += w * x0 * x0;
  B.d01 += w * x0 * x1;
  B.d02 += w * x0 * x2;
  B.d11 += w * x1 * x1;
  B.d12 += w * x1 * x2;
  B.d22 += w * x2 * x2;
}

// Schur complement inverse in FP64: out = (alpha, g0..2, G00 G01 G02 G11 G12 G22)
__device__ __forceinline__ void block_inverse(const Block& B, double* out) {
  double ia = 1.0 / B.a;
  double bt0 = B.b0 * ia, bt1 = B.b1 * ia, bt2 = B.b2 * ia;
  double t00 = B.d00 - B.b0 * bt0, t01 = B.d01 - B.b0 * bt1, t02 = B.d02 - B.b0 * bt2;
  double t11 = B.d11 - B.b1 * bt1, t12 = B.d12 - B.b1 * bt2, t22 = B.d22 - B.b2 * bt2;
  double c00 = t11 * t22 - t12 * t12, c01 = t02 * t12 - t01 * t22, c02 = t01 * t12 - t02 * t11;
  double c11 = t00 * t22 - t02 * t02, c12 = t01 * t02 - t00 * t12, c22 = t00 * t11 - t01 * t01;
  double idet = 1.0 / (t00 * c00 + t01 * c01 + t02 * c02);
  double G00 = c00 * idet, G01 = c01 * idet, G02 = c02 * idet;
  double G11 = c11 * idet, G12 = c12 * idet, G22 = c22 * idet;
  double g0 = G00 * bt0 + G01 * bt1 + G02 * bt2;
  double g1 = G01 * bt0 + G11 * bt1 + G12 * bt2;
  double g2 = G02 * bt0 + G12 * bt1 + G22 * bt2;
  out[0] = ia + bt0 * g0 + bt1 * g1 + bt2 * g2;
  out[1] = g0;
  out[2] = g1;
  out[3] = g2;
  out[4] = G00;
  out[5] = G01;
  out[6] = G02;
  out[7] = G11;
  out[8] = G12;
  out[9] = G22;
}

// dq = H^{-1} r with the factor f = (alpha, g, G); r = (r_c[3], r_a[9])
template <typename T, typename F>
__device__ __forceinline__ void block_apply(const F* f, const T* r, T* dq) {
  const T al = (T)f[0], g0 = (T)f[1], g1 = (T)f[2], g2 = (T)f[3];
  const T G00 = (T)f[4], G01 = (T)f[5], G02 = (T)f[6], G11 = (T)f[7], G12 = (T)f[8],
          G22 = (T)f[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T* ra = r + 3 + 3 * k;
    dq[k] = al * r[k] - (g0 * ra[0] + g1 * ra[1] + g2 * ra[2]);
    dq[3 + 3 * k + 0] = -g0 * r[k] + G00 * ra[0] + G01 * ra[1] + G02 * ra[2];
    dq[3 + 3 * k + 1] = -g1 * r[k] + G01 * ra[0] + G11 * ra[1] + G12 * ra[2];
    dq[3 + 3 * k + 2] = -g2 * r[k] + G02 * ra[0] + G12 * ra[1] + G22 * ra[2];
  }
}

// q^{k+1/2} = q^k + H^{-1} r in place: each entry one fused chain that starts
// from its own value (in FP32 the low position word, which carries the
// displacement within the step), so the increment is never formed apart
template <typename T, typename F>
__device__ __forceinline__ void block_apply_add(const F* f, const T* r, T* q) {
  constexpr int L = sizeof(T) == 4 ? 12 : 0;
  const T al = (T)f[0], g0 = (T)f[1], g1 = (T)f[2], g2 = (T)f[3];
  const T G00 = (T)f[4], G01 = (T)f[5], G02 = (T)f[6], G11 = (T)f[7], G12 = (T)f[8],
          G22 = (T)f[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T* ra = r + 3 + 3 * k;
    q[L + k] = fma(al, r[k], fma(-g2, ra[2], fma(-g1, ra[1], fma(-g0, ra[0], q[L + k]))));
    T* a = q + 3 + 3 * k;
    a[0] = fma(G02, ra[2], fma(G01, ra[1], fma(G00, ra[0], fma(-g0, r[k], a[0]))));
    a[1] = fma(G12, ra[2], fma(G11, ra[1], fma(G01, ra[0], fma(-g1, r[k], a[1]))));
    a[2] = fma(G22, ra[2], fma(G12, ra[1], fma(G02, ra[0], fma(-g2, r[k], a[2]))));
  }
}

// r += J(x)^T f : r_c += f, r_a[k] += f_k x
template <typename T>
__device__ __forceinline__ void add_JT(T* r, const T* x, T f0, T f1, T f2) {
  r[0] += f0;
  r[1] += f1;
  r[2] += f2;
  r[3] += f0 * x[0];
  r[4] += f0 * x[1];
  r[5] += f0 * x[2];
  r[6] += f1 * x[0];
  r[7] += f1 * x[1];
  r[8] += f1 * x[2];
  r[9] += f2 * x[0];
  r[10] += f2 * x[1];
  r[11] += f2 * x[2];
}

// ---- positions: plain in FP64, compensated pair c_hi + c_lo in FP32 ----------

// d = c_a - c_b
template <typename T>
__device__ __forceinline__ void pos_diff(const T* qa, const T* qb, T* d) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if constexpr (sizeof(T) == 4)
      d[k] = (qa[k] - qb[k]) + (qa[12 + k] - qb[12 + k]);
    else
      d[k] = qa[k] - qb[k];
  }
}

// c += dc within a step: in FP32 the increment goes to the low word only, so the
// high word stays the step's starting position and the low word carries the
// displacement (small, hence exact to a few 1e-9 m); pos_renorm folds it back
// at the end of the step
template <typename T>
__device__ __forceinline__ void pos_add_lo(T* q, T d0, T d1, T d2) {
  constexpr int L = sizeof(T) == 4 ? 12 : 0;
  q[L] += d0;
  q[L + 1] += d1;
  q[L + 2] += d2;
}

// (hi, lo) <- two-sum of hi + lo (FP32); nothing to do in FP64
template <typename T>
__device__ __forceinline__ void pos_renorm(T* q) {
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T hi = q[k], lo = q[12 + k];
      const T s = hi + lo;
      const T bv = s - hi;
      q[12 + k] = (hi - (s - bv)) + (lo - bv);
      q[k] = s;
    }
  }
}

template <typename T>
__device__ __forceinline__ double pos_value(const T* q, int k) {
  if constexpr (sizeof(T) == 4)
    return (double)q[k] + (double)q[12 + k];
  else
    return (double)q[k];
}

// bond vector d = y_o - y_s = (c_o - c_s) + A_o x_o - A_s x_s; world partner
// (qo == nullptr): y_o = x_o.  Each component is one fused chain that starts
// from the difference of the high position words and ends with the low words'.
template <typename T>
__device__ __forceinline__ void bond_vec(const T* qs, const T* xs, const T* qo, const T* xo, T* d) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const T* as = qs + 3 + 3 * r;
    T u;
    if (qo) {
      const T* ao = qo + 3 + 3 * r;
      u = qo[r] - qs[r];
      u = fma(ao[0], xo[0], u);
      u = fma(ao[1], xo[1], u);
      u = fma(ao[2], xo[2], u);
    } else {
      u = xo[r] - qs[r];
    }
    u = fma(-as[0], xs[0], u);
    u = fma(-as[1], xs[1], u);
    u = fma(-as[2], xs[2], u);
    if constexpr (sizeof(T) == 4) u += qo ? qo[12 + r] - qs[12 + r] : -qs[12 + r];
    d[r] = u;
  }
}

// The part of the bond point y = c + A x that changes within a step: in FP32 the
// low word c_lo + A x (the high word c_hi of the body position stays fixed
// through a step), in FP64 all of y.  One fused chain per component.
template <typename T>
__device__ __forceinline__ void bond_point_part(const T* q, const T* x, T* y) {
  constexpr int L = sizeof(T) == 4 ? 12 : 0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const T* a = q + 3 + 3 * r;
    y[r] = fma(a[2], x[2], fma(a[1], x[1], fma(a[0], x[0], q[L + r])));
  }
}

// r += M (s - q): translational block m I, three affine blocks Pi (sym)
template <typename T>
__device__ __forceinline__ void add_inertia(T* r, const T* mass, const T* s, const T* q) {
  const T m = mass[0], p00 = mass[1], p01 = mass[2], p02 = mass[3], p11 = mass[4],
          p12 = mass[5], p22 = mass[6];
  T dsq[3];
  pos_diff(s, q, dsq);
  r[0] += m * dsq[0];
  r[1] += m * dsq[1];
  r[2] += m * dsq[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T d0 = s[3 + 3 * k] - q[3 + 3 * k], d1 = s[4 + 3 * k] - q[4 + 3 * k],
      d2 = s[5 + 3 * k] - q[5 + 3 * k];
    r[3 + 3 * k] += p00 * d0 + p01 * d1 + p02 * d2;
    r[4 + 3 * k] += p01 * d0 + p11 * d1 + p12 * d2;
    r[5 + 3 * k] += p02 * d0 + p12 * d1 + p22 * d2;
  }
}

// The constant part of the inertia term when s stays fixed through a step's
// iterations: ms = M s, so that M (s - q) = ms - M q costs one fused chain per
// component.  In FP32 only the low position words enter: the caller keeps the
// high words of q equal to those of s through the iterations (increments go to
// the low word), so m (c_s - c_q) = m lo_s - m lo_q.
template <typename T>
__device__ __forceinline__ void mass_times(const T* mass, const T* s, T* ms) {
  constexpr int L = sizeof(T) == 4 ? 12 : 0;
  const T m = mass[0], p00 = mass[1], p01 = mass[2], p02 = mass[3], p11 = mass[4],
          p12 = mass[5], p22 = mass[6];
#pragma unroll
  for (int c = 0; c < 3; ++c) ms[c] = m * s[L + c];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T a0 = s[3 + 3 * k], a1 = s[4 + 3 * k], a2 = s[5 + 3 * k];
    ms[3 + 3 * k] = p00 * a0 + p01 * a1 + p02 * a2;
    ms[4 + 3 * k] = p01 * a0 + p11 * a1 + p12 * a2;
    ms[5 + 3 * k] = p02 * a0 + p12 * a1 + p22 * a2;
  }
}

// r = ms - M q (the inertia term M (s - q) with ms = M s from mass_times): the
// diagonal of Pi first, then, with offdiag, its off-diagonal entries.  A caller
// whose bodies all have a diagonal Pi (boxes and spheres in their own frames)
// passes offdiag = false: the terms it skips are products with zero, so the
// result is the same.
template <typename T>
__device__ __forceinline__ void inertia_from(T* r, const T* mass, const T* ms, const T* q, bool offdiag) {
  constexpr int L = sizeof(T) == 4 ? 12 : 0;
  const T m = mass[0], p00 = mass[1], p01 = mass[2], p02 = mass[3], p11 = mass[4],
          p12 = mass[5], p22 = mass[6];
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = fma(-m, q[L + c], ms[c]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[3 + 3 * k] = fma(-p00, q[3 + 3 * k], ms[3 + 3 * k]);
    r[4 + 3 * k] = fma(-p11, q[4 + 3 * k], ms[4 + 3 * k]);
    r[5 + 3 * k] = fma(-p22, q[5 + 3 * k], ms[5 + 3 * k]);
  }
  if (offdiag) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T a0 = q[3 + 3 * k], a1 = q[4 + 3 * k], a2 = q[5 + 3 * k];
      r[3 + 3 * k] = fma(-p02, a2, fma(-p01, a1, r[3 + 3 * k]));
      r[4 + 3 * k] = fma(-p12, a2, fma(-p01, a0, r[4 + 3 * k]));
      r[5 + 3 * k] = fma(-p12, a1, fma(-p02, a0, r[5 + 3 * k]));
    }
  }
}

// q^T M q of a 12-component vector whose position part c is given apart,
// formed in the arithmetic type (one body's share) and handed over in FP64 for
// the sums across bodies
template <typename T>
__device__ __forceinline__ double m_norm2(const T* mass, const T* c, const T* q) {
  const T m = mass[0], p00 = mass[1], p01 = mass[2], p02 = mass[3], p11 = mass[4],
          p12 = mass[5], p22 = mass[6];
  T s = m * (c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T a0 = q[3 + 3 * k], a1 = q[4 + 3 * k], a2 = q[5 + 3 * k];
    s += a0 * (p00 * a0 + p01 * a1 + p02 * a2) + a1 * (p01 * a0 + p11 * a1 + p12 * a2) +
         a2 * (p02 * a0 + p12 * a1 + p22 * a2);
  }
  return (double)s;
}

}  // namespace pabd
