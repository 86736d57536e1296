// kernels_tile.h -- the batched substep: one workgroup owns a tile of up to TB
// bodies made of whole scenes (joint scenes without contacts), and runs the
// complete step of Algorithm 1 for them -- prediction, K global/local Jacobi
// iterations, velocity recovery -- with the bodies' q^k and the points of
// their bond ends exchanged through LDS (double-buffered: one barrier per
// iteration).  Tiles never interact, so one launch runs nsteps consecutive
// steps of its tiles: a body's data is loaded once per launch, and its q and v
// are stored after every step.  The grid is persistent: workgroups stride over
// the device tile table, so the captured graph's launch shape does not depend
// on which scenes are resident.
#pragma once

#include "common.h"
#include "device_math.h"
#include "kernels_step.h"

namespace pabd {

struct TileTable {
  const int* first;    // first body of the tile
  const int* count;    // bodies in the tile (including released holes)
  const int* kmax;     // largest K among the tile's scenes
  const int* n_tiles;  // device count of tiles
};

// LDS layout of one q buffer of a tile: the first four values of every
// record (the position words, in FP32 the high ones, and A_00) in slots of CS
// values, then the rest of every record (the other entries of A and, in FP32,
// the low position words) in slots of RS values.  The splits keep register
// quads aligned, and the slot sizes (16 and 48 bytes in FP32, 48 and 80 in
// FP64) put the 16-byte accesses of eight neighbouring lanes in distinct
// banks.  A bond point slot is YS values.
template <typename T>
struct TileLds {
  static constexpr bool F32 = sizeof(T) == 4;
  static constexpr int QR = Rec<T>::Q;
  static constexpr int CS = F32 ? 4 : 6;
  static constexpr int RN = QR - 4;  // record values after the first four
  static constexpr int RS = F32 ? 12 : 10;
  static constexpr int YS = F32 ? 4 : 6;
  __device__ static int rest(int tb, int slot) { return (tb + 1) * CS + RS * slot; }
  __device__ static void put(T* buf, int tb, int slot, const T* q) {
    store<T, 4>(buf + CS * slot, q);
    store<T, RN>(buf + rest(tb, slot), q + 4);
  }
  __device__ static void get(const T* buf, int tb, int slot, T* q) {
    load<T, 4>(buf + CS * slot, q);
    load<T, RN>(buf + rest(tb, slot), q + 4);
  }
};

template <typename T, int TB, int MAXE>
__global__ void __launch_bounds__(TB, sizeof(T) == 4 ? 3 : 1) k_tile_step(View<T> v, TileTable tt, int nsteps) {
  constexpr int QR = Rec<T>::Q;
  using L = TileLds<T>;
  // q^k of the tile's bodies (double-buffered) plus, in slot TB, a still body
  // at the origin (c = 0, A = I), the partner of an end anchored in the world.
  // A buffer holds the position words of all slots, then the rest of each
  // record (TileLds).
  __shared__ T lq[2][(TB + 1) * (L::CS + L::RS)];
  // the bond points of each body's first MAXE ends at q^k, double-buffered
  // like q, end by end: y = c + A x, in FP32 its low part c_lo + A x (the high
  // part is the body's c_hi).  An end whose partner publishes the mirror end
  // (the other end of the same bond) takes the partner's point from here.
  __shared__ T ly[2][MAXE * TB * L::YS];
  const int lane = threadIdx.x;
  const int ntiles = *tt.n_tiles;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int first = tt.first[t], nb = tt.count[t], kmax = tt.kmax[t];
    const int i = first + lane;
    const int scn = lane < nb ? v.bscene[i] : -1;
    if (lane < L::CS) {  // (0, 0, 0, A_00 = 1)
      lq[0][TB * L::CS + lane] = lane == 3 ? (T)1 : (T)0;
      lq[1][TB * L::CS + lane] = lane == 3 ? (T)1 : (T)0;
    }
    if (lane < L::RS) {  // A_01 .. A_22 of the identity, then zeros
      const T o = (lane == 3 || lane == 7) ? (T)1 : (T)0;
      lq[0][L::rest(TB, TB) + lane] = o;
      lq[1][L::rest(TB, TB) + lane] = o;
    }
    // what no step changes is loaded once per launch; q and v stay in
    // registers from step to step and are written back after every step
    const bool pinned = scn >= 0 && (v.flags[i] & F_PINNED);
    T q[QR], vw[VW], m[MW], fac[FW];
    // per register end: the bond point x in the body frame, h^2 kappa, h^2
    // phi^-, the partner's slot in lq and the offset in ly of the point of its
    // mirror end
    T X[MAXE][3], kap[MAXE], phim[MAXE];
    int qslot[MAXE], yoff[MAXE];
    bool mirrored[MAXE], some_unmirrored[MAXE];
#pragma unroll
    for (int u = 0; u < MAXE; ++u) {
      mirrored[u] = false;
      qslot[u] = TB;
      yoff[u] = L::YS * (u * TB + lane);  // own point: an address in range for ends read the long way
    }
    int e0 = 0, ne = 0;
    if (scn >= 0) {
      load<T, QR>(v.qn + (size_t)QR * i, q);
      // a pinned body publishes its bond points too, for its partners
      e0 = v.srow[i];
      ne = v.srow_end[i] - e0;
#pragma unroll
      for (int u = 0; u < MAXE; ++u) {
        if (u < ne) {
          T Eu[EW];
          load<T, EW>(v.se + (size_t)EW * (e0 + u), Eu);
          X[u][0] = Eu[0];
          X[u][1] = Eu[1];
          X[u][2] = Eu[2];
          kap[u] = Eu[3];
          phim[u] = Eu[7];
          const int p = v.se_partner[e0 + u];
          qslot[u] = p < 0 ? TB : p - first;
          if (p >= 0 && !pinned) {
            // the mirror end: the bonds between two bodies have their ends in
            // bond order on both sides, so the end that is the n-th of this
            // body towards p pairs with the n-th end of p towards this body
            int rank = 0;
#pragma unroll
            for (int w = 0; w < u; ++w) rank += qslot[w] == qslot[u] ? 1 : 0;
            const int b0 = v.srow[p], b1 = min(v.srow_end[p], b0 + MAXE);
#pragma unroll
            for (int w = 0; w < MAXE; ++w)
              if (b0 + w < b1 && !mirrored[u] && v.se_partner[b0 + w] == i) {
                if (rank == 0) {
                  mirrored[u] = true;
                  yoff[u] = L::YS * (w * TB + p - first);
                }
                --rank;
              }
          }
        }
      }
      if (!pinned) {
        load<T, VW>(v.vel + (size_t)VW * i, vw);
        load<T, MW>(v.mass + (size_t)MW * i, m);
        load<T, FW>(v.fac + (size_t)FW * i, fac);
      } else {
        ne = min(ne, MAXE);  // a pinned body only publishes its register ends
      }
    }
    // whether every body of the wave has a diagonal Pi (boxes and spheres in
    // their own frames): the inertia term then takes the diagonal alone
    // (wave-uniform, fixed for the launch)
    const bool diag_pi = wave_all(scn < 0 || pinned || (m[2] == (T)0 && m[3] == (T)0 && m[5] == (T)0));
    // per register end, whether some lane of the wave takes it the long way
    // (wave-uniform, fixed for the launch)
#pragma unroll
    for (int u = 0; u < MAXE; ++u) some_unmirrored[u] = wave_any(!pinned && u < ne && !mirrored[u]);
    // whether some lane of the tile reads a partner's q^k from LDS after the
    // first iteration (an end taken the long way, or ends beyond the register
    // ones); when none does, q^k is published only for the first iteration,
    // where the partners' high position words are read (uniform over the
    // workgroup, whose waves read each other's slots)
    bool long_way = scn >= 0 && !pinned && ne > MAXE;
#pragma unroll
    for (int u = 0; u < MAXE; ++u) long_way = long_way || (scn >= 0 && !pinned && u < ne && !mirrored[u]);
    const bool need_q = __syncthreads_or(long_way);
    // the scene's step count, read once per launch and advanced in registers
    // beside the scene table's counter (which the scene's first lane advances
    // for the host), so that no step waits for the previous one's store
    int sstep = scn >= 0 ? v.scenes[scn].step : 0;
    for (int step = 0; step < nsteps; ++step) {
      const bool present = scn >= 0 && sstep < v.scenes[scn].steps_total;
      const bool moving = present && !pinned;
      // scene constants are re-read every step rather than held in registers
      // through the iterations
      const int K = present ? v.scenes[scn].iters : 0;
      // the residual is formed on the launch's last step and on a scene's own
      // last step (the only ones whose residual can be read afterwards)
      const bool want_rho = present && (step == nsteps - 1 || sstep + 1 >= v.scenes[scn].steps_total);
      // M s of the prediction s: the inertia term's part that no iteration
      // changes (q's high position words stay those of s through the step)
      T ms[QW];
      if (moving) {
        // prediction, in place: q becomes s
        const SceneDev& S = v.scenes[scn];
        const T h = (T)S.h;
        T As[9];
        predict_rotation(q + 3, vw + 3, h, As);
#pragma unroll
        for (int c = 0; c < 9; ++c) q[3 + c] = As[c];
        pos_add_lo(q, h * (vw[0] + h * (T)S.g0), h * (vw[1] + h * (T)S.g1), h * (vw[2] + h * (T)S.g2));
        mass_times(m, q, ms);
      }
      // v is rebuilt from q^{n+1} and q^n after the iterations: nothing of it
      // needs to live through them
#pragma unroll
      for (int c = 0; c < VW; ++c) vw[c] = (T)0;
      double num = 0.0, den = 0.0;
      T dh[MAXE][3];  // FP32: c_hi of the partner minus c_hi of this body, per end
      for (int k = 0; k < kmax; ++k) {
        T* buf = lq[k & 1];
        T* ybuf = ly[k & 1];
        if (present) {
          if (k == 0 || need_q) L::put(buf, TB, lane, q);
#pragma unroll
          for (int u = 0; u < MAXE; ++u)
            if (u < ne) {
              T y[4];
              bond_point_part(q, X[u], y);
              y[3] = (T)0;
              store<T, 4>(ybuf + L::YS * (u * TB + lane), y);
            }
        }
        __syncthreads();
        if (moving && k < K) {
          // r = M (s - q^k) + sum of the ends' J^T f (the forces carry h^2);
          // starting from the inertia term leaves no accumulator to clear
          T r[QW];
          inertia_from(r, m, ms, q, !diag_pi);
#pragma unroll
          for (int u = 0; u < MAXE; ++u)
            if (u < ne) {
              // d = y_o - y_s from the two published points; in FP32 plus the
              // difference of the high position words, fixed through the step
              // and so taken once, in its first iteration
              T ys[4], yo[4], d[3], f[3];
              load<T, 4>(ybuf + L::YS * (u * TB + lane), ys);
              load<T, 4>(ybuf + yoff[u], yo);
              if constexpr (sizeof(T) == 4) {
                if (k == 0) {
                  const T* co = buf + L::CS * qslot[u];
#pragma unroll
                  for (int c = 0; c < 3; ++c) dh[u][c] = co[c] - q[c];
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) d[c] = dh[u][c] + (yo[c] - ys[c]);
              } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) d[c] = yo[c] - ys[c];
              }
              if (some_unmirrored[u]) {
                // an end anchored in the world, or whose mirror is not among the
                // partner's register ends: from the partner's q and its record
                if (!mirrored[u]) {
                  T Eg[EW], qj[QR];
                  load<T, EW>(v.se + (size_t)EW * (e0 + u), Eg);
                  L::get(buf, TB, qslot[u], qj);
                  bond_vec<T>(q, Eg, qj, Eg + 4, d);
                }
              }
              end_force(kap[u], phim[u], d, f);
              add_JT(r, X[u], f[0], f[1], f[2]);
            }
          for (int e = e0 + MAXE; e < e0 + ne; ++e) {
            T Eg[EW];
            load<T, EW>(v.se + (size_t)EW * e, Eg);
            const int p = v.se_partner[e];
            T d[3], f[3], qj[QR];
            L::get(buf, TB, p < 0 ? TB : p - first, qj);
            bond_vec<T>(q, Eg, qj, Eg + 4, d);
            quad_end_force(Eg, d, f);
            add_JT(r, Eg, f[0], f[1], f[2]);
          }
          // q^{k+1} in place; a lane's last iteration keeps what its residual
          // |q^{k+1} - q^k|_M / |q^k|_M needs
          const bool last = k == K - 1 && want_rho;
          constexpr int LO = sizeof(T) == 4 ? 12 : 0;
          T Aold[9], cold[3];
          if (last) {
            const T cc[3] = {(T)pos_value(q, 0), (T)pos_value(q, 1), (T)pos_value(q, 2)};
            den = m_norm2(m, cc, q);
#pragma unroll
            for (int c = 0; c < 9; ++c) Aold[c] = q[3 + c];
#pragma unroll
            for (int c = 0; c < 3; ++c) cold[c] = q[LO + c];
          }
          block_apply_add(fac, r, q);
          // the rare polar continuation passes X through this lane's words of
          // the other q buffer, which no lane reads before the next iteration
          // has rewritten them
          polar_rotation_spill(q + 3, lq[(k + 1) & 1] + L::rest(TB, lane), v.polar, i);
          if (last) {
            T dd[QW];
#pragma unroll
            for (int c = 0; c < 3; ++c) dd[c] = q[LO + c] - cold[c];
#pragma unroll
            for (int c = 0; c < 9; ++c) dd[3 + c] = q[3 + c] - Aold[c];
            num = m_norm2(m, dd, dd);
          }
        }
      }
      __syncthreads();  // every lane is done with the q buffers
      // per-scene FP64 residual: each body's partials through LDS
      double* red = reinterpret_cast<double*>(&lq[0][0]);
      red[lane] = num;
      red[TB + lane] = den;
      if (moving) {
        // q^n is still the body's record in HBM, stored after the previous step
        T qn[QR];
        load<T, QR>(v.qn + (size_t)QR * i, qn);
        recover_velocity(q, qn, (T)(1.0 / v.scenes[scn].h), vw);
        bool finite = true;
#pragma unroll
        for (int c = 0; c < QR; ++c) finite = finite && isfinite(q[c]);
#pragma unroll
        for (int c = 0; c < 6; ++c) finite = finite && isfinite(vw[c]);
        if (!finite) atomicOr(v.health + scn, 1);
        pos_renorm(q);
        store<T, QR>(v.qn + (size_t)QR * i, q);
        store<T, VW>(v.vel + (size_t)VW * i, vw);
      }
      // pairwise sums over the scene's bodies by their index within the scene:
      // the same order wherever the scene sits in the tile (skipped on the
      // steps where no scene of the tile forms its residual)
      const int loc = present ? i - v.scenes[scn].body_off : 1;
      const int nbs = present ? v.scenes[scn].n_bodies : 0;
      if (__syncthreads_or(want_rho)) {
#pragma unroll
        for (int w = 1; w < TB; w <<= 1) {
          if ((loc & (2 * w - 1)) == 0 && loc + w < nbs) {
            red[lane] += red[lane + w];
            red[TB + lane] += red[TB + lane + w];
          }
          __syncthreads();
        }
      }
      if (present && loc == 0) {
        if (want_rho) {
          const double a = red[lane], b = red[TB + lane];
          v.rho[scn] = b > 0.0 ? sqrt(a / b) : 0.0;
        }
        v.scenes[scn].step = sstep + 1;
      }
      if (present) ++sstep;
      __syncthreads();  // LDS settled for the next step or tile
    }
  }
}

}  // namespace pabd
