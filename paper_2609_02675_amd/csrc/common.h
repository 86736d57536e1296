// common.h -- device data layout of the PABD library.
//
// Per-body records are packed arrays of structures so one body is a few 16-byte
// vector loads (a bond partner's coordinates are gathered by its neighbours):
//   Q    12 T : c0 c1 c2 | a1 (3) | a2 (3) | a3 (3)      (A rows)
//        (FP32: 16 floats, c_lo0 c_lo1 c_lo2 kc appended, see Rec; kc =
//        round(scale * free mass), the body's share of a contact's h^2 kappa)
//   VEL   8 T : v0 v1 v2 w0 w1 w2 - -
//   MASS  8 T : m  Pi00 Pi01 Pi02 Pi11 Pi12 Pi22 -
//   FAC  12 T : alpha g0 g1 g2 G00 G01 G02 G11 G12 G22 - -   (H^{-1}, FP64-computed)
//   BLK  10 double : a b0 b1 b2 D00 D01 D02 D11 D12 D22     (static part of H)
// Static bond ends (two per bond between bodies, one per world bond) are a CSR
// over bodies in (body, bond id) order:
//   END   8 T : xs0 xs1 xs2 kappa xo0 xo1 xo2 phim   (phim = phi^- = -kappa l)
//   plus the partner body (int, -1 = world; xo then in world coordinates).
// Contact ends live in fixed per-body slots (capacity C per body, ELL by body):
//   CEND FP64 12 T : xs0 xs1 xs2 kappa xo0 xo1 xo2 mu n0 n1 n2 -
//   CEND FP32  8 T : xs0 xs1 xs2 nu xo0 xo1 xo2 nv   (n in octahedral form;
//        kappa is the larger kc of the two q records, mu the scene's)
//   plus partner (int) and a 64-bit sort key; n is oriented for the owning side
//   (it points from the partner's surface towards the owner).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pabd {

constexpr int QW = 12, VW = 8, MW = 8, FW = 12, EW = 8, CW = 12;

// Stored width of a contact end record: CW values in FP64, 8 in FP32.
template <typename T>
struct ContactRec {
  static constexpr int W = sizeof(T) == 4 ? 8 : CW;
};

// Stored width of a Q record.  In FP32 the body position is kept as an
// unevaluated sum c_hi + c_lo of two floats (c_lo at 12..14) so that bond
// vectors between bodies far from the origin keep FP32 relative accuracy (the
// joint gap is millimetres on positions of tens of metres); FP64 needs no
// compensation.
template <typename T>
struct Rec {
  static constexpr int Q = 12;
};
template <>
struct Rec<float> {
  static constexpr int Q = 16;
};
constexpr uint8_t F_PINNED = 1, F_NOCONTACT = 2;
constexpr uint8_t F_VARIABLE = 4;  // set by the library: the body owns ends whose weight changes every iteration
// kind of a variable end, held in the last of its four per-end values: > 0 an
// augmented end (that value is kappa_start), -p a polynomial end of even order p,
// and the two odd codes below the two ends of a slider bond (never an order)
constexpr int AL_SLIDER_POINT = -1;  // the point side: drawn to the foot on the partner's line
constexpr int AL_SLIDER_LINE = -3;   // the line side: its foot point drawn to the partner's point

// per-scene parameters (device scene table)
struct SceneDev {
  double h, g0, g1, g2;
  double t0;
  double kscale, margin, mu;
  double al_beta, al_alpha, al_gamma;  // augmented-bond constants
  double cell;      // broad-phase cell size of the current step
  int iters;
  int body_off, n_bodies;
  int plane_off, n_planes;
  int contact;      // collision detection enabled
  int ccap;         // contact ends per body
  int step;         // completed steps
  int debug;        // bit0: skip the local step (single scenes on the flat path only)
  int steps_total;  // the scene is frozen once step reaches this
  int tiled;        // advanced by the tile kernel (which also reduces its residual)
  int ce_off;       // first contact slot of the scene: body b of the scene owns
                    // slots ce_off + (b - body_off) * ccap ... + ccap - 1
  int resident;     // advanced by the resident step kernel (whole steps from LDS)
  int pad;
};

// first contact slot of body i of scene S
__device__ __forceinline__ size_t ce_base(const SceneDev& S, int i) {
  return (size_t)S.ce_off + (size_t)(i - S.body_off) * (size_t)S.ccap;
}

// A contact end as the narrow phase stages it, in the order its atomics give:
// the end's record, its partner and its sort key (partner + 1, feature, side)
// side by side, so that staging an end writes one run of bytes (48 in FP32)
// and the sort reads one.
template <typename T>
struct alignas(16) StageRec {
  T C[ContactRec<T>::W];
  int partner;
  int pad;
  unsigned long long key;
};
static_assert(sizeof(StageRec<float>) == 48, "an FP32 staged end is one 48-byte run");

template <typename T>
struct View {
  int n;  // bodies covered by the arrays
  T* q[2];
  T* qn;
  T* vel;
  T* s;
  const T* mass;
  T* fac;
  double* blk;
  const uint8_t* flags;
  const uint8_t* shape;
  const T* half;  // 4 per body: hx hy hz radius
  const int* group;
  const int* bscene;
  // static ends
  const int* srow;      // first static end of the body
  const int* srow_end;  // one past its last static end
  const int* se_partner;
  T* se;
  // 4 per end for ends whose weight changes every iteration: augmented
  // (kappa_j, lambda_j, l, kappa_start > 0), polynomial (kappa, 0, l, -p), else 0
  T* al;
  const double* se64;  // 4 per end: xs (3), kappa in FP64 (for the factorisation)
  // contacts
  int* ccount;
  int* ce_partner;
  unsigned long long* ce_key;
  T* ce;
  // narrow-phase output before the canonical sort, one record per end
  StageRec<T>* ce_stage;
  const double* planes;
  // residual partials
  double* r_num;
  double* r_den;
  // scenes
  SceneDev* scenes;
  int* health;  // per scene: bit0 non-finite, bit1 contact overflow
  double* rho;  // per scene: residual of the last iteration of the last step
  // per body, 2 each: local steps whose rotation came from the SVD, and those
  // whose input had det <= 0
  unsigned* polar;
};

// ---- vector load/store of packed records --------------------------------------

template <typename T, int N>
__device__ __forceinline__ void ld(const T* p, T* out);
template <typename T, int N>
__device__ __forceinline__ void st(T* p, const T* in);

template <int N>
__device__ __forceinline__ void ld_f(const float* p, float* out) {
#pragma unroll
  for (int k = 0; k < N / 4; ++k) {
    float4 v = reinterpret_cast<const float4*>(p)[k];
    out[4 * k] = v.x;
    out[4 * k + 1] = v.y;
    out[4 * k + 2] = v.z;
    out[4 * k + 3] = v.w;
  }
}
template <int N>
__device__ __forceinline__ void ld_d(const double* p, double* out) {
#pragma unroll
  for (int k = 0; k < N / 2; ++k) {
    double2 v = reinterpret_cast<const double2*>(p)[k];
    out[2 * k] = v.x;
    out[2 * k + 1] = v.y;
  }
}
template <int N>
__device__ __forceinline__ void st_f(float* p, const float* in) {
#pragma unroll
  for (int k = 0; k < N / 4; ++k)
    reinterpret_cast<float4*>(p)[k] = make_float4(in[4 * k], in[4 * k + 1], in[4 * k + 2], in[4 * k + 3]);
}
template <int N>
__device__ __forceinline__ void st_d(double* p, const double* in) {
#pragma unroll
  for (int k = 0; k < N / 2; ++k)
    reinterpret_cast<double2*>(p)[k] = make_double2(in[2 * k], in[2 * k + 1]);
}

template <typename T, int N>
__device__ __forceinline__ void load(const T* p, T* out) {
  if constexpr (sizeof(T) == 4)
    ld_f<N>(reinterpret_cast<const float*>(p), reinterpret_cast<float*>(out));
  else
    ld_d<N>(reinterpret_cast<const double*>(p), reinterpret_cast<double*>(out));
}
template <typename T, int N>
__device__ __forceinline__ void store(T* p, const T* in) {
  if constexpr (sizeof(T) == 4)
    st_f<N>(reinterpret_cast<float*>(p), reinterpret_cast<const float*>(in));
  else
    st_d<N>(reinterpret_cast<double*>(p), reinterpret_cast<const double*>(in));
}

}  // namespace pabd
