// engine.h -- device storage for a set of scenes and the launch sequence of one
// step over it.  Used by the plain scene handle (one scene, one kernel launch
// per iteration, captured into a graph) and by the batch (flat kernels for
// scenes that need contacts or do not fit a tile; tile kernel for the rest).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "host_scene.h"
#include "kernels_contact.h"
#include "kernels_flat.h"
#include "kernels_resident.h"
#include "kernels_step.h"
#include "kernels_tile.h"

namespace pabd {

#define PABD_HIP(x)                                                        \
  do {                                                                     \
    hipError_t e_ = (x);                                                   \
    if (e_ != hipSuccess) {                                                \
      err = std::string(#x) + " failed: " + hipGetErrorString(e_);         \
      return PABD_E_DEVICE;                                                \
    }                                                                      \
  } while (0)

// device memory: hipMalloc/hipFree, or a caller's allocator (pabd_set_allocator);
// each engine keeps the one in force when it was created, for its whole life
struct DeviceAllocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*release)(void*, void*) = nullptr;
  void* ctx = nullptr;
  hipError_t get(void** p, size_t bytes) const {
    if (alloc) {
      *p = alloc(bytes, ctx);
      return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
  }
  void put(void* p) const {
    if (!p) return;
    if (alloc) {
      if (release) release(p, ctx);
    } else {
      (void)hipFree(p);
    }
  }
};

inline DeviceAllocator& current_allocator() {
  static DeviceAllocator a;
  return a;
}

// one segment of a staged upload: bytes at src_off of the staging buffer go to dst
struct Seg {
  char* dst;
  unsigned long long src_off, bytes;
};

// copy every segment of a staged upload to its destination (segment = blockIdx.y);
// words where both ends are 4-byte aligned, bytes otherwise
__global__ void __launch_bounds__(256) k_scatter(const char* src, const Seg* segs) {
  const Seg sg = segs[blockIdx.y];
  const char* s = src + sg.src_off;
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  const unsigned long long t0 = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
  if ((((unsigned long long)sg.dst | sg.src_off | sg.bytes) & 3ull) == 0) {
    const unsigned* w = reinterpret_cast<const unsigned*>(s);
    unsigned* d = reinterpret_cast<unsigned*>(sg.dst);
    for (unsigned long long k = t0; k < sg.bytes / 4; k += stride) d[k] = w[k];
  } else {
    for (unsigned long long k = t0; k < sg.bytes; k += stride) sg.dst[k] = s[k];
  }
}

struct Caps {
  int n = 0, e = 0, s = 0, p = 0, dr = 0;
  int nc = -1;        // bodies [0, nc) may have contacts (-1: all n)
  long long cslots = 0;  // contact slots, shared by the contact scenes (SceneDev::ce_off)
  bool contacts = false;
};


template <typename T>
struct Engine {
  Caps cap;
  // per body
  T *qn = nullptr, *q0 = nullptr, *q1 = nullptr, *s = nullptr, *vel = nullptr, *mass = nullptr,
    *fac = nullptr, *half = nullptr;
  double *blk = nullptr, *mass64 = nullptr, *r_num = nullptr, *r_den = nullptr;
  uint8_t *flags = nullptr, *shape = nullptr;
  int *group = nullptr, *bscene = nullptr, *srow = nullptr, *srow_end = nullptr;
  // static ends
  int* se_partner = nullptr;
  T* se = nullptr;
  T* al = nullptr;
  double* se64 = nullptr;
  // contacts
  int *ccount = nullptr, *ce_partner = nullptr;
  unsigned long long *ce_key = nullptr, *reach = nullptr;
  T* ce = nullptr;
  StageRec<T>* ce_stage = nullptr;
  int *bucket_count = nullptr, *bucket_start = nullptr, *bucket_fill = nullptr, *scan_tmp = nullptr;
  int *hist = nullptr, *large = nullptr, *counters = nullptr, *ltask = nullptr;
  double* breach = nullptr;
  BroadRec* brec = nullptr;
  int2* pairs = nullptr;
  int tb = 0, pcap = 0, ncb = 0;
  // scenes
  SceneDev* scenes = nullptr;
  int* health = nullptr;
  double* rho = nullptr;
  unsigned* polar = nullptr;  // 2 per body (View::polar)
  double* planes = nullptr;
  // driven bonds
  int *drv_scene = nullptr, *drv_end_i = nullptr, *drv_end_j = nullptr;
  double* drv_param = nullptr;
  // residual history (optional)
  double *rh_num = nullptr, *rh_den = nullptr, *rh_rho = nullptr;
  int rh_k = 0;
  // scenes run by the resident step kernel: [0] contact scenes (four lanes per
  // body), [1] the others; capacity one entry per scene slot, counts on the device
  int* res_list[2] = {nullptr, nullptr};
  int* res_count = nullptr;
  bool res_variable = true;  // some resident scene has variable ends
  // flat-path schedule: lanes that share a contact body's ends (1, 2, 4, 8 or
  // 16) and wavefronts per workgroup of the iteration launches (1, 2 or 4)
  int contact_lanes = 4, group_waves = 1;

  std::vector<void*> allocs;
  std::string err;
  DeviceAllocator dev = current_allocator();
  // staged uploads: one pinned host buffer, one device buffer, grown on demand
  char* h_stage = nullptr;
  char* d_stage = nullptr;
  size_t stage_cap = 0;
  // upload with one plain copy per array instead (no pinned or device staging
  // buffer: for an engine whose memory must not grow)
  bool direct_upload = false;

  ~Engine() { release(); }
  void release() {
    for (void* p : allocs) dev.put(p);
    allocs.clear();
    if (h_stage) (void)hipHostFree(h_stage);
    dev.put(d_stage);
    h_stage = d_stage = nullptr;
    stage_cap = 0;
  }

  struct Put {
    void* dst;
    const void* src;
    size_t bytes;
  };

  // every put in one host-to-device copy plus one scatter launch; returns when done
  pabd_status staged_upload(const std::vector<Put>& puts, hipStream_t st) {
    if (direct_upload) {
      for (const Put& p : puts)
        if (p.bytes) PABD_HIP(hipMemcpyAsync(p.dst, p.src, p.bytes, hipMemcpyHostToDevice, st));
      PABD_HIP(hipStreamSynchronize(st));
      return PABD_OK;
    }
    size_t total = 0;
    std::vector<Seg> segs;
    for (const Put& p : puts) {
      if (!p.bytes) continue;
      segs.push_back(Seg{static_cast<char*>(p.dst), (unsigned long long)total, (unsigned long long)p.bytes});
      total += (p.bytes + 15) / 16 * 16;
    }
    if (segs.empty()) return PABD_OK;
    const size_t need = total + segs.size() * sizeof(Seg);
    if (need > stage_cap) {
      size_t cap2 = std::max<size_t>(need, std::max<size_t>(2 * stage_cap, 1 << 20));
      if (h_stage) (void)hipHostFree(h_stage);
      dev.put(d_stage);
      h_stage = d_stage = nullptr;
      stage_cap = 0;
      PABD_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_stage), cap2, hipHostMallocDefault));
      PABD_HIP(dev.get(reinterpret_cast<void**>(&d_stage), cap2));
      stage_cap = cap2;
    }
    size_t k = 0;
    for (const Put& p : puts) {
      if (!p.bytes) continue;
      std::memcpy(h_stage + segs[k].src_off, p.src, p.bytes);
      ++k;
    }
    std::memcpy(h_stage + total, segs.data(), segs.size() * sizeof(Seg));
    PABD_HIP(hipMemcpyAsync(d_stage, h_stage, need, hipMemcpyHostToDevice, st));
    size_t largest = 0;
    for (const Seg& g : segs) largest = std::max<size_t>(largest, g.bytes);
    const unsigned gx = (unsigned)std::min<size_t>(1024, std::max<size_t>(1, (largest / 4 + 255) / 256));
    hipLaunchKernelGGL(k_scatter, dim3(gx, (unsigned)segs.size()), dim3(256), 0, st, (const char*)d_stage,
                       reinterpret_cast<const Seg*>(d_stage + total));
    PABD_HIP(hipGetLastError());
    PABD_HIP(hipStreamSynchronize(st));
    return PABD_OK;
  }

  template <typename U>
  pabd_status alloc(U*& p, size_t count) {
    void* v = nullptr;
    hipError_t e = dev.get(&v, std::max<size_t>(count, 1) * sizeof(U));
    if (e != hipSuccess) {
      err = std::string("device allocation of ") + std::to_string(count * sizeof(U)) +
            " bytes failed: " + hipGetErrorString(e);
      (void)hipGetLastError();
      return PABD_E_OOM;
    }
    allocs.push_back(v);
    p = static_cast<U*>(v);
    return PABD_OK;
  }

#define PABD_TRY(x)                      \
  do {                                   \
    pabd_status st_ = (x);               \
    if (st_ != PABD_OK) return st_;      \
  } while (0)

  pabd_status allocate(const Caps& c) {
    cap = c;
    const size_t n = c.n;
    constexpr int QR = Rec<T>::Q;
    PABD_TRY(alloc(qn, QR * n));
    PABD_TRY(alloc(q0, QR * n));
    PABD_TRY(alloc(q1, QR * n));
    PABD_TRY(alloc(s, QR * n));
    PABD_TRY(alloc(vel, VW * n));
    PABD_TRY(alloc(mass, MW * n));
    PABD_TRY(alloc(fac, FW * n));
    PABD_TRY(alloc(half, 4 * n));
    PABD_TRY(alloc(blk, 10 * n));
    PABD_TRY(alloc(mass64, 8 * n));
    PABD_TRY(alloc(r_num, n));
    PABD_TRY(alloc(r_den, n));
    PABD_TRY(alloc(flags, n));
    PABD_TRY(alloc(shape, n));
    PABD_TRY(alloc(group, n));
    PABD_TRY(alloc(bscene, n));
    PABD_TRY(alloc(srow, n));
    PABD_TRY(alloc(srow_end, n));
    PABD_TRY(alloc(se_partner, (size_t)c.e));
    PABD_TRY(alloc(se, EW * (size_t)c.e));
    PABD_TRY(alloc(al, 4 * (size_t)c.e));
    PABD_TRY(alloc(se64, 4 * (size_t)c.e));
    PABD_TRY(alloc(ccount, n));
    PABD_TRY(alloc(scenes, (size_t)c.s));
    PABD_TRY(alloc(health, (size_t)c.s));
    PABD_TRY(alloc(polar, 2 * n));
    PABD_TRY(alloc(rho, (size_t)c.s));
    PABD_TRY(alloc(reach, (size_t)c.s));
    PABD_TRY(alloc(planes, 4 * (size_t)c.p));
    PABD_TRY(alloc(drv_scene, (size_t)c.dr));
    PABD_TRY(alloc(drv_end_i, (size_t)c.dr));
    PABD_TRY(alloc(drv_end_j, (size_t)c.dr));
    PABD_TRY(alloc(drv_param, 13 * (size_t)c.dr));
    PABD_TRY(alloc(res_list[0], (size_t)c.s));
    PABD_TRY(alloc(res_list[1], (size_t)c.s));
    PABD_TRY(alloc(res_count, 2));
    if (c.contacts) {
      ncb = c.nc < 0 ? c.n : std::min(c.nc, c.n);
      const size_t nb = (size_t)ncb, nc = (size_t)std::max(1LL, c.cslots);
      PABD_TRY(alloc(ce, ContactRec<T>::W * nc));
      PABD_TRY(alloc(ce_partner, nc));
      PABD_TRY(alloc(ce_key, nc));
      PABD_TRY(alloc(ce_stage, nc));
      // power of two, at most 2^20 so the three-pass scan (1024 x 1024) covers it
      tb = 1024;
      while (tb < 2 * ncb && tb < (1 << 20)) tb <<= 1;
      PABD_TRY(alloc(bucket_count, (size_t)tb));
      PABD_TRY(alloc(bucket_start, (size_t)tb + 1));
      PABD_TRY(alloc(bucket_fill, (size_t)tb));
      PABD_TRY(alloc(scan_tmp, (size_t)(tb / 1024 + 2)));
      PABD_TRY(alloc(brec, nb));
      PABD_TRY(alloc(breach, nb));
      PABD_TRY(alloc(large, nb));
      PABD_TRY(alloc(ltask, nb + 1));
      PABD_TRY(alloc(counters, 3));
      PABD_TRY(alloc(hist, (size_t)REACH_BINS * c.s));
      // candidate pairs: half a pair per slot, at least 16 per body
      const size_t pc = std::max(nb * 16, nc / 2);
      if (pc > (size_t)INT_MAX) {
        err = "candidate pair capacity exceeds 2^31";
        return PABD_E_INVALID;
      }
      pcap = (int)pc;
      PABD_TRY(alloc(pairs, pc));
    }
    // every body slot starts unused
    std::vector<int> neg(n, -1);
    PABD_HIP(hipMemcpy(bscene, neg.data(), n * sizeof(int), hipMemcpyHostToDevice));
    std::vector<int> zero(std::max<size_t>(n, (size_t)c.s) + 1, 0);
    PABD_HIP(hipMemcpy(srow, zero.data(), n * sizeof(int), hipMemcpyHostToDevice));
    PABD_HIP(hipMemcpy(srow_end, zero.data(), n * sizeof(int), hipMemcpyHostToDevice));
    PABD_HIP(hipMemcpy(ccount, zero.data(), n * sizeof(int), hipMemcpyHostToDevice));
    PABD_HIP(hipMemcpy(health, zero.data(), (size_t)c.s * sizeof(int), hipMemcpyHostToDevice));
    const int zero_counts[2] = {0, 0};
    PABD_HIP(hipMemcpy(res_count, zero_counts, sizeof zero_counts, hipMemcpyHostToDevice));
    std::vector<double> rz((size_t)c.s, 0.0);
    PABD_HIP(hipMemcpy(rho, rz.data(), rz.size() * sizeof(double), hipMemcpyHostToDevice));
    std::vector<unsigned> zero2n(2 * n, 0u);
    PABD_HIP(hipMemcpy(polar, zero2n.data(), zero2n.size() * sizeof(unsigned), hipMemcpyHostToDevice));
    std::vector<int> dneg(std::max(1, c.dr), -1);
    PABD_HIP(hipMemcpy(drv_scene, dneg.data(), dneg.size() * sizeof(int), hipMemcpyHostToDevice));
    std::vector<double> dz(n, 0.0);
    PABD_HIP(hipMemcpy(r_num, dz.data(), n * sizeof(double), hipMemcpyHostToDevice));
    PABD_HIP(hipMemcpy(r_den, dz.data(), n * sizeof(double), hipMemcpyHostToDevice));
    return PABD_OK;
  }

  View<T> view() const {
    View<T> v{};
    v.n = cap.n;
    v.q[0] = q0;
    v.q[1] = q1;
    v.qn = qn;
    v.vel = vel;
    v.s = s;
    v.mass = mass;
    v.fac = fac;
    v.blk = blk;
    v.flags = flags;
    v.shape = shape;
    v.half = half;
    v.group = group;
    v.bscene = bscene;
    v.srow = srow;
    v.srow_end = srow_end;
    v.se_partner = se_partner;
    v.se = se;
    v.al = al;
    v.se64 = se64;
    v.ccount = ccount;
    v.ce_partner = ce_partner;
    v.ce_key = ce_key;
    v.ce = ce;
    v.ce_stage = ce_stage;
    v.planes = planes;
    v.r_num = r_num;
    v.r_den = r_den;
    v.scenes = scenes;
    v.health = health;
    v.polar = polar;
    v.rho = rho;
    return v;
  }

  template <typename U>
  pabd_status put(U* dst, const U* src, size_t count, hipStream_t st) {
    if (!count) return PABD_OK;
    PABD_HIP(hipMemcpyAsync(dst, src, count * sizeof(U), hipMemcpyHostToDevice, st));
    return PABD_OK;
  }

  // Upload a prepared scene at body offset boff, end offset eoff, plane offset
  // poff, driven offset doff into scene slot sidx.
  pabd_status upload(const HostScene& hs, int boff, int eoff, int poff, int doff, int sidx,
                     hipStream_t st) {
    const size_t n = hs.n, ne = hs.ne;
    constexpr int QR = Rec<T>::Q;
    std::vector<T> tq(QR * n, (T)0), tv(VW * n), tm(MW * n), th(4 * n), te(EW * ne);
    for (size_t b = 0; b < n; ++b) {
      for (int k = 0; k < QW; ++k) tq[QR * b + k] = (T)hs.qn[QW * b + k];
      if (QR > QW) {  // compensated position: c = c_hi + c_lo
        for (int k = 0; k < 3; ++k)
          tq[QR * b + 12 + k] = (T)(hs.qn[QW * b + k] - (double)tq[QR * b + k]);
        // the body's share of a contact's h^2 kappa, round(scale * free mass)
        const double mfree = (hs.flags[b] & F_PINNED) ? 0.0 : hs.mass64[8 * b];
        tq[QR * b + Q_KAPPA] = (T)(hs.params.kscale * mfree);
      }
    }
    for (size_t k = 0; k < VW * n; ++k) tv[k] = (T)hs.vel[k];
    for (size_t b = 0; b < n; ++b) {
      const double* M = &hs.mass64[8 * b];
      // packed sym Pi: 00 01 02 11 12 22 (mass64 stores Pi00 Pi01 Pi02 Pi11 Pi12 Pi22 at 1..6)
      for (int k = 0; k < 8; ++k) tm[MW * b + k] = (T)M[k];
    }
    for (size_t k = 0; k < 4 * n; ++k) th[k] = (T)hs.half[k];
    // bond records carry h^2 kappa and h^2 phi^- (the iteration sums h^2-scaled forces)
    const double h2 = hs.params.h * hs.params.h;
    for (size_t k = 0; k < EW * ne; ++k) te[k] = (T)((k % EW == 3 || k % EW == 7) ? h2 * hs.se[k] : hs.se[k]);
    std::vector<T> ta(4 * ne);
    for (size_t k = 0; k < 4 * ne; ++k) ta[k] = (T)hs.al[k];
    std::vector<int> part(ne), rows(n), rows_end(n), bs(n, sidx);
    for (size_t e = 0; e < ne; ++e) part[e] = hs.se_partner[e] < 0 ? -1 : hs.se_partner[e] + boff;
    for (size_t b = 0; b < n; ++b) {
      rows[b] = hs.srow[b] + eoff;
      rows_end[b] = hs.srow[b + 1] + eoff;
    }
    std::vector<uint8_t> fl(hs.flags);
    SceneDev S = hs.params;
    S.body_off = boff;
    S.plane_off = poff;
    S.step = 0;
    std::vector<Put> puts;
    auto add = [&](auto* dst, const auto* src, size_t count) {
      puts.push_back(Put{dst, src, count * sizeof(*src)});
    };
    add(qn + QR * (size_t)boff, tq.data(), tq.size());
    add(vel + VW * (size_t)boff, tv.data(), tv.size());
    add(mass + MW * (size_t)boff, tm.data(), tm.size());
    add(mass64 + 8 * (size_t)boff, hs.mass64.data(), hs.mass64.size());
    add(half + 4 * (size_t)boff, th.data(), th.size());
    add(flags + boff, fl.data(), fl.size());
    add(shape + boff, hs.shape.data(), hs.shape.size());
    add(group + boff, hs.group.data(), hs.group.size());
    add(bscene + boff, bs.data(), bs.size());
    add(srow + boff, rows.data(), rows.size());
    add(srow_end + boff, rows_end.data(), rows_end.size());
    add(se_partner + eoff, part.data(), part.size());
    add(se + EW * (size_t)eoff, te.data(), te.size());
    add(al + 4 * (size_t)eoff, ta.data(), ta.size());
    add(se64 + 4 * (size_t)eoff, hs.se64.data(), hs.se64.size());
    add(planes + 4 * (size_t)poff, hs.planes.data(), hs.planes.size());
    add(scenes + sidx, &S, 1);
    int zero = 0;
    add(health + sidx, &zero, 1);
    std::vector<unsigned> zero_polar(2 * n, 0u);
    add(polar + 2 * (size_t)boff, zero_polar.data(), zero_polar.size());
    const double rho0 = 0.0;  // no step taken yet
    add(rho + sidx, &rho0, 1);
    const size_t nd = hs.drv_end_i.size();
    std::vector<int> di(nd), dj(nd), ds(nd, sidx);
    for (size_t k = 0; k < nd; ++k) {
      di[k] = hs.drv_end_i[k] < 0 ? -1 : hs.drv_end_i[k] + eoff;
      dj[k] = hs.drv_end_j[k] < 0 ? -1 : hs.drv_end_j[k] + eoff;
    }
    if (nd) {
      add(drv_scene + doff, ds.data(), nd);
      add(drv_end_i + doff, di.data(), nd);
      add(drv_end_j + doff, dj.data(), nd);
      add(drv_param + 13 * (size_t)doff, hs.drv_param.data(), hs.drv_param.size());
    }
    return staged_upload(puts, st);
  }

  // mark body slots [boff, boff + n) and driven entries [doff, doff + nd) unused
  pabd_status clear_bodies(int boff, int n, hipStream_t st, int doff = 0, int nd = 0) {
    std::vector<int> neg(std::max(n, nd), -1);
    PABD_TRY(put(bscene + boff, neg.data(), (size_t)n, st));
    if (nd > 0) PABD_TRY(put(drv_scene + doff, neg.data(), (size_t)nd, st));
    PABD_HIP(hipStreamSynchronize(st));
    return PABD_OK;
  }

  static dim3 grid_for(int n, int bs) { return dim3((unsigned)std::max(1, (n + bs - 1) / bs)); }

  // contact-bond construction for every contact scene among the bodies
  // [0, min(cap.n, contact bodies))
  // a single contact scene of at most this many bodies takes the all-pairs broad
  // phase (at most 2.1M pair threads)
  static constexpr int BRUTE_MAX = 2048;
  // predict: the prep kernel also runs the step's prediction for the bodies
  // [0, min(cap.n, contact bodies))
  void launch_contacts(int n_scenes, hipStream_t st, bool predict = false) {
    View<T> v = view();
    v.n = std::min(cap.n, ncb);
    ContactBuf cb{tb,    bucket_count, bucket_start, bucket_fill, brec,  reach,   hist,
                  breach, large,       counters,     pairs,       pcap,  mass64,  scan_tmp, ltask};
    const int n = v.n;
    const bool brute = n_scenes == 1 && n <= BRUTE_MAX;
    const int nbk = brute ? 0 : tb;  // bucket counts cleared by the prep kernel
    hipLaunchKernelGGL(k_contact_prep<T>, grid_for(std::max({n, REACH_BINS * n_scenes, nbk}), 256), dim3(256), 0,
                       st, v, cb, n_scenes, nbk, predict);
    hipLaunchKernelGGL(k_contact_reach<T>, grid_for(n, 256), dim3(256), 0, st, v, cb);
    if (brute) {
      // one scene of few bodies: all pairs directly, no spatial hash
      const long long threads = (long long)n + (long long)n * (n - 1) / 2;
      hipLaunchKernelGGL(k_broad_brute<T>, dim3((unsigned)std::max(1LL, (threads + 255) / 256)), dim3(256), 0, st,
                         v, cb, 0, n);
    } else {
      hipLaunchKernelGGL(k_contact_cells, grid_for(n_scenes, 64), dim3(64), 0, st, scenes, n_scenes,
                         (const unsigned long long*)reach, (const int*)hist);
      hipLaunchKernelGGL(k_hash_count<T>, grid_for(n, 256), dim3(256), 0, st, v, cb);
      const int nb = (tb + 1023) / 1024;
      hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(1024), 0, st, (const int*)bucket_count,
                         bucket_start, tb, scan_tmp);
      hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, scan_tmp, nb, bucket_start + tb);
      hipLaunchKernelGGL(k_scan_add, grid_for(tb, 256), dim3(256), 0, st, bucket_start, tb,
                         (const int*)scan_tmp);
      hipLaunchKernelGGL(k_hash_fill<T>, grid_for(n, 256), dim3(256), 0, st, v, cb);
      hipLaunchKernelGGL(k_broad_small<T>, grid_for((int)std::min<long long>((long long)n * BLPB, INT_MAX), 256),
                         dim3(256), 0, st, v, cb);
      hipLaunchKernelGGL(k_large_tasks<T>, dim3(1), dim3(1024), 0, st, v, cb);
      hipLaunchKernelGGL(k_broad_large<T>, dim3(1024), dim3(BL_CHUNK), 0, st, v, cb);
    }
    const int ng = std::min(8192, std::max(1, (pcap + 255) / 256));
    hipLaunchKernelGGL(k_narrow_pairs<T>, dim3(ng), dim3(256), 0, st, v, cb);
    hipLaunchKernelGGL(k_sort_contacts<T>, dim3((unsigned)std::max(1, n)), dim3(64), 0, st, v);
  }

  // the scene slots the resident step kernel runs: [0] contact scenes, [1] others
  // variable: some listed scene has variable ends (augmented, polynomial, slider)
  pabd_status set_resident(const std::vector<int>& contact, const std::vector<int>& other, bool variable,
                           hipStream_t st) {
    res_variable = variable;
    const int counts[2] = {(int)contact.size(), (int)other.size()};
    if (counts[0]) PABD_HIP(hipMemcpyAsync(res_list[0], contact.data(), counts[0] * sizeof(int), hipMemcpyHostToDevice, st));
    if (counts[1]) PABD_HIP(hipMemcpyAsync(res_list[1], other.data(), counts[1] * sizeof(int), hipMemcpyHostToDevice, st));
    PABD_HIP(hipMemcpyAsync(res_count, counts, sizeof counts, hipMemcpyHostToDevice, st));
    PABD_HIP(hipStreamSynchronize(st));
    return PABD_OK;
  }

  // one step of the resident scenes: grid[0] workgroups over the contact list,
  // grid[1] over the other (extents rounded by the caller; extra workgroups leave)
  // n_driven > 0: the resident scenes' driven anchors and refactor run inside
  // the resident kernel (no flat-path scene shares the step)
  void launch_resident(const int* grid, int n_driven, hipStream_t st) {
    View<T> v = view();
    const DrivenTable dt{n_driven, drv_scene, drv_end_i, drv_end_j, drv_param, mass64};
    const bool driven = n_driven > 0;
    if (res_variable && driven)
      launch_resident_as<2, true>(v, grid, dt, st);
    else if (res_variable)
      launch_resident_as<2, false>(v, grid, dt, st);
    else if (driven)
      launch_resident_as<1, true>(v, grid, dt, st);
    else
      launch_resident_as<1, false>(v, grid, dt, st);
  }
  template <int ENDS, bool DRIVEN>
  void launch_resident_as(const View<T>& v, const int* grid, const DrivenTable& dt, hipStream_t st) {
    if (grid[0] > 0)
      hipLaunchKernelGGL((k_resident_step<T, 4, true, ENDS, DRIVEN>), dim3(grid[0]), dim3(Resident<T>::NT), 0,
                         st, v, (const int*)res_list[0], (const int*)res_count, dt);
    if (grid[1] > 0)
      hipLaunchKernelGGL((k_resident_step<T, 1, false, ENDS, DRIVEN>), dim3(grid[1]), dim3(Resident<T>::NT), 0,
                         st, v, (const int*)res_list[1], (const int*)(res_count + 1), dt);
  }

  // FP64 block factorisation of bodies [first, first + count)
  void launch_factor(hipStream_t st, int first = 0, int count = -1) {
    if (count < 0) count = cap.n;
    if (count == 0) return;
    hipLaunchKernelGGL(k_factor<T>, grid_for(count, 256), dim3(256), 0, st, view(),
                       (const double*)mass64, first, count);
  }

  // the K iteration launches of a flat step, CL lanes per contact body; by
  // default one wavefront per workgroup, so that a small scene's waves spread
  // over as many CUs (and L1 caches) as there are waves
  template <int CL>
  void launch_iterations(int kmax, bool contacts, bool history, hipStream_t st, const FlatWave* waves,
                         const int* n_waves, int wave_grid, double* hn, double* hd) {
    View<T> v = view();
    const int gw = group_waves;
    const dim3 wg(64 * gw);
    const dim3 gc = grid_for((int)std::min<long long>((long long)cap.n * CL, INT_MAX), 64 * gw);
    const dim3 g1 = grid_for(cap.n, 64 * gw);
    const dim3 gwv((unsigned)std::max(1, (wave_grid + gw - 1) / gw));
    for (int k = 0; k < kmax; ++k) {
      if (waves && !history)
        hipLaunchKernelGGL((k_iterate_waves<T, CL>), gwv, wg, 0, st, v, k, waves, n_waves);
      else if (contacts)
        hipLaunchKernelGGL((k_iterate<T, true, CL>), gc, wg, 0, st, v, k, hn, hd);
      else
        hipLaunchKernelGGL((k_iterate<T, false, 1>), g1, wg, 0, st, v, k, hn, hd);
    }
  }

  // One step of Algorithm 1 with flat per-body kernels (one launch per iteration).
  // With a wave table (batches), the iterations run over it instead:
  // contact_lanes lanes per body of a contact scene, one per body of any other
  // scene.
  //
  // resident_grid (optional): the scenes of the resident lists take their whole
  // step in the resident kernel, after the contact construction; with
  // flat = false no flat-path kernel is launched (every flat scene is resident).
  void launch_flat_step(int n_scenes, int kmax, bool contacts, int n_driven, bool history,
                        bool finish_scenes, hipStream_t st, const FlatWave* waves = nullptr,
                        const int* n_waves = nullptr, int wave_grid = 0,
                        const int* resident_grid = nullptr, bool flat = true) {
    View<T> v = view();
    const dim3 g = grid_for(cap.n, 256), b(256);
    // with every scene resident the driven update and refactor run in the
    // resident kernel, after the contact construction, which reads neither
    const bool drive_inside = resident_grid && !flat;
    if (n_driven > 0 && !drive_inside) {
      hipLaunchKernelGGL(k_update_driven<T>, grid_for(n_driven, 64), dim3(64), 0, st, v, n_driven,
                         (const int*)drv_scene, (const int*)drv_end_i, (const int*)drv_end_j,
                         (const double*)drv_param);
      launch_factor(st);
    }
    // with contacts, the contact construction's first kernel also predicts
    // (when its body range covers the flat path's)
    const bool predict_in_prep = contacts && flat && ncb >= cap.n;
    if (contacts) launch_contacts(n_scenes, st, predict_in_prep);
    if (resident_grid) launch_resident(resident_grid, drive_inside ? n_driven : 0, st);
    if (!flat) return;
    if (!predict_in_prep) hipLaunchKernelGGL(k_predict<T>, g, b, 0, st, v);
    double* hn = history ? rh_num : nullptr;
    double* hd = history ? rh_den : nullptr;
    if (history) {
      const long long nh = (long long)kmax * cap.n;
      const dim3 gz((unsigned)std::max(1LL, (nh + 255) / 256));
      hipLaunchKernelGGL(k_zero_double, gz, dim3(256), 0, st, rh_num, nh);
      hipLaunchKernelGGL(k_zero_double, gz, dim3(256), 0, st, rh_den, nh);
    }
    switch (contact_lanes) {
      case 1: launch_iterations<1>(kmax, contacts, history, st, waves, n_waves, wave_grid, hn, hd); break;
      case 2: launch_iterations<2>(kmax, contacts, history, st, waves, n_waves, wave_grid, hn, hd); break;
      case 8: launch_iterations<8>(kmax, contacts, history, st, waves, n_waves, wave_grid, hn, hd); break;
      case 16: launch_iterations<16>(kmax, contacts, history, st, waves, n_waves, wave_grid, hn, hd); break;
      default: launch_iterations<4>(kmax, contacts, history, st, waves, n_waves, wave_grid, hn, hd); break;
    }
    // (each body's step ends in its last iteration: velocities, health, q^{n+1})
    if (!finish_scenes) return;
    // the residual and the end of the step (step counters) of the flat-path scenes
    hipLaunchKernelGGL(k_reduce_residual, dim3(std::max(1, n_scenes)), dim3(RED_THREADS), 0, st, scenes,
                       n_scenes, (const double*)r_num, (const double*)r_den, rho);
    if (history)
      hipLaunchKernelGGL(k_reduce_history, dim3(std::max(1, kmax)), dim3(256), 0, st, cap.n, kmax,
                         (const double*)rh_num, (const double*)rh_den, rh_rho);
  }
};

}  // namespace pabd
