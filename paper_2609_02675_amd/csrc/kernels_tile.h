// kernels_tile.h -- the batched substep: one workgroup owns a tile of up to TB
// bodies made of whole scenes (joint scenes without contacts), and runs the
// complete step of Algorithm 1 for them -- prediction, K global/local Jacobi
// iterations, velocity recovery -- with the bodies' q^k exchanged through LDS
// (double-buffered: one barrier per iteration).  Tiles never interact, so one
// launch runs nsteps consecutive steps of its tiles: a body's data is loaded
// once per launch, and its q and v are stored after every step.  The grid is
// persistent: workgroups stride over the device tile table, so the captured
// graph's launch shape does not depend on which scenes are resident.
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

template <typename T, int TB, int MAXE>
__global__ void __launch_bounds__(TB, sizeof(T) == 4 ? 3 : 1) k_tile_step(View<T> v, TileTable tt, int nsteps) {
  constexpr int QR = Rec<T>::Q;
  // q^k of the tile's bodies (double-buffered) plus, in slot TB, a still body
  // at the origin (c = 0, A = I): an end anchored in the world takes it as its
  // partner, so every end runs the same code
  __shared__ T lq[2][(TB + 1) * QR];
  __shared__ T lqn[TB * QR];  // q^n of each lane's body, for velocity recovery
  const int lane = threadIdx.x;
  const int ntiles = *tt.n_tiles;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int first = tt.first[t], nb = tt.count[t], kmax = tt.kmax[t];
    const int i = first + lane;
    const int scn = lane < nb ? v.bscene[i] : -1;
    if (lane < QR) {
      const T o = (lane == 3 || lane == 7 || lane == 11) ? (T)1 : (T)0;
      lq[0][TB * QR + lane] = o;
      lq[1][TB * QR + lane] = o;
    }
    // what no step changes is loaded once per launch; q and v stay in
    // registers from step to step and are written back after every step
    const bool pinned = scn >= 0 && (v.flags[i] & F_PINNED);
    T q[QR], vw[VW], m[MW], fac[FW];
    T E[MAXE][EW];
    int part[MAXE];
    int e0 = 0, ne = 0;
    if (scn >= 0) {
      load<T, QR>(v.qn + (size_t)QR * i, q);
      if (!pinned) {
        load<T, VW>(v.vel + (size_t)VW * i, vw);
        load<T, MW>(v.mass + (size_t)MW * i, m);
        load<T, FW>(v.fac + (size_t)FW * i, fac);
        e0 = v.srow[i];
        ne = v.srow_end[i] - e0;
#pragma unroll
        for (int u = 0; u < MAXE; ++u)
          if (u < ne) {
            load<T, EW>(v.se + (size_t)EW * (e0 + u), E[u]);
            const int p = v.se_partner[e0 + u];
            part[u] = p < 0 ? TB : p - first;
          }
      }
    }
    for (int step = 0; step < nsteps; ++step) {
      // the scene's step counter was advanced by its first lane before the
      // previous step's last barrier
      const bool present = scn >= 0 && v.scenes[scn].step < v.scenes[scn].steps_total;
      const bool moving = present && !pinned;
      // scene constants are re-read every step rather than held in registers
      // through the iterations
      const int K = present ? v.scenes[scn].iters : 0;
      // M s of the prediction s: the inertia term's part that no iteration
      // changes (q's high position words stay those of s through the step)
      T ms[QW];
      if (moving) {
        store<T, QR>(lqn + QR * lane, q);
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
      for (int k = 0; k < kmax; ++k) {
        T* buf = lq[k & 1];
        if (present) store<T, QR>(buf + QR * lane, q);
        __syncthreads();
        if (moving && k < K) {
          // r = M (s - q^k) + sum of the ends' J^T f (the forces carry h^2);
          // starting from the inertia term leaves no accumulator to clear
          T r[QW];
          inertia_from(r, m, ms, q);
#pragma unroll
          for (int u = 0; u < MAXE; ++u)
            if (u < ne) {
              T d[3], f[3], qj[QR];
              load<T, QR>(buf + QR * part[u], qj);
              bond_vec<T>(q, E[u], qj, E[u] + 4, d);
              quad_end_force(E[u], d, f);
              add_JT(r, E[u], f[0], f[1], f[2]);
            }
          for (int e = e0 + MAXE; e < e0 + ne; ++e) {
            T Eg[EW];
            load<T, EW>(v.se + (size_t)EW * e, Eg);
            const int p = v.se_partner[e];
            T d[3], f[3], qj[QR];
            load<T, QR>(buf + QR * (p < 0 ? TB : p - first), qj);
            bond_vec<T>(q, Eg, qj, Eg + 4, d);
            quad_end_force(Eg, d, f);
            add_JT(r, Eg, f[0], f[1], f[2]);
          }
          T dq[QW];
          block_apply(fac, r, dq);
          // q^{k+1} in place; a lane's last iteration keeps what its residual
          // |q^{k+1} - q^k|_M / |q^k|_M needs (the position part of the
          // difference is the increment itself)
          const bool last = k == K - 1;
          T Aold[9];
          if (last) {
            const double cc[3] = {pos_value(q, 0), pos_value(q, 1), pos_value(q, 2)};
            den = m_norm2(m, cc, q);
#pragma unroll
            for (int c = 0; c < 9; ++c) Aold[c] = q[3 + c];
          }
          pos_add_lo(q, dq[0], dq[1], dq[2]);
#pragma unroll
          for (int c = 0; c < 9; ++c) q[3 + c] += dq[3 + c];
          // the rare polar continuation passes X through this lane's words of
          // the other q buffer, which no lane reads before the next iteration
          // has rewritten them
          polar_rotation_spill(q + 3, lq[(k + 1) & 1] + QR * lane);
          if (last) {
            T dd[QW];
#pragma unroll
            for (int c = 0; c < 3; ++c) dd[c] = dq[c];
#pragma unroll
            for (int c = 0; c < 9; ++c) dd[3 + c] = q[3 + c] - Aold[c];
            const double dc[3] = {(double)dq[0], (double)dq[1], (double)dq[2]};
            num = m_norm2(m, dc, dd);
          }
        }
      }
      __syncthreads();  // every lane is done with the q buffers
      // per-scene FP64 residual: each body's partials through LDS
      double* red = reinterpret_cast<double*>(&lq[0][0]);
      red[lane] = num;
      red[TB + lane] = den;
      if (moving) {
        T qn[QR];
        load<T, QR>(lqn + QR * lane, qn);
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
      __syncthreads();
      // pairwise sums over the scene's bodies by their index within the scene:
      // the same order wherever the scene sits in the tile
      const int loc = present ? i - v.scenes[scn].body_off : 1;
      const int nbs = present ? v.scenes[scn].n_bodies : 0;
#pragma unroll
      for (int w = 1; w < TB; w <<= 1) {
        if ((loc & (2 * w - 1)) == 0 && loc + w < nbs) {
          red[lane] += red[lane + w];
          red[TB + lane] += red[TB + lane + w];
        }
        __syncthreads();
      }
      if (present && loc == 0) {
        const double a = red[lane], b = red[TB + lane];
        v.rho[scn] = b > 0.0 ? sqrt(a / b) : 0.0;
        v.scenes[scn].step += 1;
      }
      __syncthreads();  // LDS and step counters settled for the next step or tile
    }
  }
}

}  // namespace pabd
