// kernels_step.h -- per-body kernels of one step of Algorithm 1 over a flat range
// of bodies that may belong to several scenes (scene table lookup per body):
//   k_predict   prediction loop (v* = v + h g, c* = c + h v*, A* = R(dQ) A^n; q^0 = s)
//   k_factor    FP64 block H_i = M_i + h^2 sum w J^T J (Sec. 4.2.1) and its sparse
//               inverse (Sec. 4.3), stored as the FP64 block and a T factor
//   (the iterations themselves are in kernels_flat.h)
//   k_reduce_residual  per-scene FP64 residual, fixed summation order, and the
//               end of the scene's step
#pragma once

#include "common.h"
#include "device_math.h"

namespace pabd {

// the prediction of body i (Algorithm 1): s = q^0 from q^n and the velocities,
// and the augmented ends' warm start; scenes of the resident kernel, finished
// scenes and unused slots are left alone
template <typename T>
__device__ __forceinline__ void predict_body(const View<T>& v, int i) {
  constexpr int QR = Rec<T>::Q;
  const int sc = v.bscene[i];
  if (sc < 0) return;
  T q[QR];
  load<T, QR>(v.qn + (size_t)QR * i, q);
  if (v.scenes[sc].step >= v.scenes[sc].steps_total || v.scenes[sc].resident) return;
  if (v.flags[i] & F_PINNED) {
    store<T, QR>(v.q[0] + (size_t)QR * i, q);
    store<T, QR>(v.q[1] + (size_t)QR * i, q);
    store<T, QR>(v.s + (size_t)QR * i, q);
    return;
  }
  const SceneDev& S = v.scenes[sc];
  const T h = (T)S.h;
  T vw[VW];
  load<T, VW>(v.vel + (size_t)VW * i, vw);
  T s[QR];
#pragma unroll
  for (int c = 0; c < QR; ++c) s[c] = q[c];
  pos_add_lo(s, h * (vw[0] + h * (T)S.g0), h * (vw[1] + h * (T)S.g1), h * (vw[2] + h * (T)S.g2));
  predict_rotation(q + 3, vw + 3, h, s + 3);
  store<T, QR>(v.s + (size_t)QR * i, s);
  store<T, QR>(v.q[0] + (size_t)QR * i, s);
  if (v.flags[i] & F_VARIABLE) {
    // augmented ends, warm start (Sec. 5.2.2): kappa = max(gamma kappa, kappa_start),
    // lambda = alpha gamma lambda
    const T ga = (T)S.al_gamma, ag = (T)(S.al_alpha * S.al_gamma);
    for (int e = v.srow[i]; e < v.srow_end[i]; ++e) {
      T* a = v.al + 4 * (size_t)e;
      if (!(a[3] > (T)0)) continue;  // augmented ends only
      a[0] = fmax(ga * a[0], a[3]);
      a[1] = ag * a[1];
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_predict(View<T> v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < v.n) predict_body(v, i);
}

// mass64: 8 doubles per body (m, Pi sym 6, -)
template <typename T>
__device__ __forceinline__ void factor_body(const View<T>& v, const double* mass64, int i) {
  const int sc = v.bscene[i];
  if (sc < 0 || (v.flags[i] & F_PINNED)) return;
  const double h2 = v.scenes[sc].h * v.scenes[sc].h;
  const double* m = mass64 + 8 * (size_t)i;
  Block B{m[0], 0, 0, 0, m[1], m[2], m[3], m[4], m[5], m[6]};
  for (int e = v.srow[i]; e < v.srow_end[i]; ++e) {
    const double* x = v.se64 + 4 * (size_t)e;
    block_add_end(B, h2 * x[3], x[0], x[1], x[2]);
  }
  double* bo = v.blk + 10 * (size_t)i;
  bo[0] = B.a; bo[1] = B.b0; bo[2] = B.b1; bo[3] = B.b2; bo[4] = B.d00;
  bo[5] = B.d01; bo[6] = B.d02; bo[7] = B.d11; bo[8] = B.d12; bo[9] = B.d22;
  double f[10];
  block_inverse(B, f);
  T ft[FW];
#pragma unroll
  for (int k = 0; k < 10; ++k) ft[k] = (T)f[k];
  ft[10] = ft[11] = (T)0;
  store<T, FW>(v.fac + (size_t)FW * i, ft);
}
template <typename T>
__global__ void __launch_bounds__(256) k_factor(View<T> v, const double* mass64, int first, int count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int i = first + t;
  if (i >= v.n) return;
  factor_body(v, mass64, i);
}

// contribution of one quadratic bond end with bond vector d = y_o - y_s, scaled
// by h^2 (the record holds h^2 kappa and h^2 phi^-):
// h^2 f = h^2 kappa d + h^2 phim d/|d| (phi^+ / d = kappa implicit, phi^- explicit)
template <typename T>
__device__ __forceinline__ void end_force(T kap, T phim, const T* d, T* f) {
  f[0] = kap * d[0];
  f[1] = kap * d[1];
  f[2] = kap * d[2];
  if (phim != (T)0) {
    T dn2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (dn2 > (T)1e-24) {
      T sc = phim * rsqrt_(dn2);
      f[0] += sc * d[0];
      f[1] += sc * d[1];
      f[2] += sc * d[2];
    }
  }
}
template <typename T>
__device__ __forceinline__ void quad_end_force(const T* E, const T* d, T* f) {
  end_force(E[3], E[7], d, f);
}

// velocity recovery from q^{n+1} (= qf) and q^n (= q0), shared with the tile kernel
template <typename T>
__device__ __forceinline__ void recover_velocity(const T* qf, const T* q0, T ih, T* vw) {
  T dc[3];
  pos_diff(qf, q0, dc);
  vw[0] = dc[0] * ih;
  vw[1] = dc[1] * ih;
  vw[2] = dc[2] * ih;
  // W = (A^{n+1} - A^n) (A^n)^T / h (A^n orthogonal: inverse = transpose)
  T dA[9], W[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) dA[c] = qf[3 + c] - q0[3 + c];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      W[3 * r + c] = dA[3 * r] * q0[3 + 3 * c] + dA[3 * r + 1] * q0[4 + 3 * c] +
                     dA[3 * r + 2] * q0[5 + 3 * c];
  // average of [w]_x and -[w]_x^T
  vw[3] = (T)0.5 * (W[7] - W[5]) * ih;
  vw[4] = (T)0.5 * (W[2] - W[6]) * ih;
  vw[5] = (T)0.5 * (W[3] - W[1]) * ih;
  vw[6] = vw[7] = (T)0;
}

// one block per scene; rho = sqrt(sum num / sum den) over the scene's bodies in a
// fixed order (strided partial sums, then a tree), so results are reproducible
constexpr int RED_THREADS = 1024;

// per flat-path scene: the FP64 residual of its last iteration, then the end of
// its step (the step counter advances unless the scene has taken all its steps)
__global__ void __launch_bounds__(RED_THREADS) k_reduce_residual(SceneDev* scenes, int n_scenes,
                                                                const double* num, const double* den,
                                                                double* rho) {
  __shared__ double sn[RED_THREADS], sd[RED_THREADS];
  const int sc = blockIdx.x;
  if (sc >= n_scenes) return;
  if (scenes[sc].tiled || scenes[sc].resident) return;  // those kernels reduce their own scenes
  const int off = scenes[sc].body_off, nb = scenes[sc].n_bodies;
  // each thread sums a fixed stride of the scene's bodies in order; the unrolled
  // loop keeps several loads in flight
  double a = 0.0, b = 0.0;
#pragma unroll 8
  for (int t = threadIdx.x; t < nb; t += RED_THREADS) {
    a += num[off + t];
    b += den[off + t];
  }
  sn[threadIdx.x] = a;
  sd[threadIdx.x] = b;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sn[threadIdx.x] += sn[threadIdx.x + w];
      sd[threadIdx.x] += sd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    rho[sc] = sd[0] > 0.0 ? sqrt(sn[0] / sd[0]) : 0.0;
    if (scenes[sc].step < scenes[sc].steps_total) scenes[sc].step += 1;
  }
}

// zero n doubles (a kernel, so that it can sit in a captured graph)
__global__ void __launch_bounds__(256) k_zero_double(double* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// residual history: rho_k for every k of the last step (plain path diagnostics);
// the partials of bodies that do not iterate (pinned) stay at the zero the step
// starts from
__global__ void __launch_bounds__(256) k_reduce_history(int n, int K, const double* num,
                                                       const double* den, double* rho) {
  __shared__ double sn[256], sd[256];
  const int k = blockIdx.x;
  if (k >= K) return;
  double a = 0.0, b = 0.0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    a += num[(size_t)k * n + t];
    b += den[(size_t)k * n + t];
  }
  sn[threadIdx.x] = a;
  sd[threadIdx.x] = b;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sn[threadIdx.x] += sn[threadIdx.x + w];
      sd[threadIdx.x] += sd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) rho[k] = sd[0] > 0.0 ? sqrt(sn[0] / sd[0]) : 0.0;
}

// driven bonds: the j-side anchor of bond b is base rotated about the axis through
// pivot by theta(t) = theta0 + amp sin(2 pi f t + phase), t = time at the end of
// the step being taken.  Updates the i-side end's partner anchor and the j-side
// end's own anchor (T and FP64 copies).
template <typename T>
__device__ __forceinline__ void update_driven_entry(const View<T>& v, int b, int sc, const int* d_end_i,
                                                    const int* d_end_j, const double* d_param) {
  const SceneDev& S = v.scenes[sc];
  if (S.step >= S.steps_total) return;
  const double t = S.t0 + (double)(S.step + 1) * S.h;
  const double* p = d_param + 13 * (size_t)b;
  const double th = p[9] + p[10] * sin(2.0 * 3.14159265358979323846 * p[11] * t + p[12]);
  const double u0 = p[0], u1 = p[1], u2 = p[2];
  const double r0 = p[6] - p[3], r1 = p[7] - p[4], r2 = p[8] - p[5];
  const double c = cos(th), s = sin(th), ud = u0 * r0 + u1 * r1 + u2 * r2;
  const double x0 = p[3] + r0 * c + (u1 * r2 - u2 * r1) * s + u0 * ud * (1 - c);
  const double x1 = p[4] + r1 * c + (u2 * r0 - u0 * r2) * s + u1 * ud * (1 - c);
  const double x2 = p[5] + r2 * c + (u0 * r1 - u1 * r0) * s + u2 * ud * (1 - c);
  const int ei = d_end_i[b], ej = d_end_j[b];
  if (ei >= 0) {
    T* E = v.se + (size_t)EW * ei;
    E[4] = (T)x0;
    E[5] = (T)x1;
    E[6] = (T)x2;
  }
  if (ej >= 0) {
    T* E = v.se + (size_t)EW * ej;
    E[0] = (T)x0;
    E[1] = (T)x1;
    E[2] = (T)x2;
    double* e64 = const_cast<double*>(v.se64) + 4 * (size_t)ej;
    e64[0] = x0;
    e64[1] = x1;
    e64[2] = x2;
  }
}
template <typename T>
__global__ void k_update_driven(View<T> v, int n_driven, const int* d_scene, const int* d_end_i,
                                const int* d_end_j, const double* d_param) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_driven) return;
  const int sc = d_scene[b];
  if (sc < 0) return;  // unused table entry
  update_driven_entry(v, b, sc, d_end_i, d_end_j, d_param);
}

}  // namespace pabd
