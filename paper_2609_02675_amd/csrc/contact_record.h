// contact_record.h -- the per-end contact record as the iterations read it.
//
// FP64: x_s (3), h^2 kappa_c, x_o (3), mu, n (3), pad: CW = 12 values.
// FP32: x_s (3), n_u, x_o (3), n_v: 8 values, 32 bytes, two 16-byte loads.
//   - The normal is stored in octahedral form (n_u, n_v): n / |n|_1 folded onto
//     the upper half of the octahedron.  It decodes to n within a few float
//     roundings, everywhere on the sphere.
//   - h^2 kappa_c = scale * max(m_i, m_j) over the pair's free masses (0 for a
//     pinned body or a plane).  It is the larger of the two bodies'
//     round(scale * m), which every FP32 q record carries in its last word:
//     rounding is monotone, so the larger rounded value is the rounded larger
//     one, and the stiffness keeps its bits.
//   - mu is the scene's.
// The FP32 iteration thus streams 32 bytes per contact end instead of 48.
#pragma once

#include "common.h"
#include "device_math.h"

namespace pabd {

// word of an FP32 q record that holds round(scale * free mass)
constexpr int Q_KAPPA = 15;

// (u, v) of a unit normal n: p = n / |n|_1, and below the equator the folded
// p_x, p_y = (1 - |p_y|) sign p_x, (1 - |p_x|) sign p_y
__host__ __device__ inline void oct_encode(const double* n, double* uv) {
  const double s = fabs(n[0]) + fabs(n[1]) + fabs(n[2]);
  double u = n[0] / s, v = n[1] / s;
  if (n[2] < 0.0) {
    const double fu = (1.0 - fabs(v)) * (u >= 0.0 ? 1.0 : -1.0);
    const double fv = (1.0 - fabs(u)) * (v >= 0.0 ? 1.0 : -1.0);
    u = fu;
    v = fv;
  }
  uv[0] = u;
  uv[1] = v;
}

// the unit normal back from (u, v): z = 1 - |u| - |v|; below the equator
// (z < 0) unfold x, y; then normalise (in FP32 with the hardware reciprocal
// square root, about 1 ulp)
template <typename T>
__device__ __forceinline__ void oct_decode(T u, T v, T* n) {
  const T z = (T)1 - fabs(u) - fabs(v);
  T x = u, y = v;
  if (z < (T)0) {
    x = ((T)1 - fabs(v)) * (u >= (T)0 ? (T)1 : (T)-1);
    y = ((T)1 - fabs(u)) * (v >= (T)0 ? (T)1 : (T)-1);
  }
  const T inv = rsqrt_(x * x + y * y + z * z);
  n[0] = x * inv;
  n[1] = y * inv;
  n[2] = z * inv;
}

// the same on the host, in FP64 (read-back of contact records)
inline void oct_decode_host(double u, double v, double* n) {
  const double z = 1.0 - fabs(u) - fabs(v);
  double x = u, y = v;
  if (z < 0.0) {
    x = (1.0 - fabs(v)) * (u >= 0.0 ? 1.0 : -1.0);
    y = (1.0 - fabs(u)) * (v >= 0.0 ? 1.0 : -1.0);
  }
  const double r = sqrt(x * x + y * y + z * z);
  n[0] = x / r;
  n[1] = y / r;
  n[2] = z / r;
}

}  // namespace pabd
