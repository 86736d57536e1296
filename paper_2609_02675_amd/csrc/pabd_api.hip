// pabd_api.hip -- the C ABI of include/pabd.h: plain scene handles and batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pabd.h"
#include "engine.h"

using namespace pabd;

namespace {

thread_local std::string g_err;

pabd_status fail(pabd_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define API_HIP(x)                                                                   \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) return fail(PABD_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool use_graphs() {
  const char* e = std::getenv("PABD_NO_GRAPH");
  return !(e && e[0] == '1');
}

// ---------------------------------------------------------------------------
// precision-erased engine interface
// ---------------------------------------------------------------------------

struct EngineBase {
  virtual ~EngineBase() = default;
  virtual pabd_status allocate(const Caps& c) = 0;
  virtual pabd_status upload(const HostScene& hs, int boff, int eoff, int poff, int doff, int sidx,
                             hipStream_t st) = 0;
  virtual pabd_status clear_bodies(int boff, int n, hipStream_t st, int doff, int nd) = 0;
  virtual void factor(hipStream_t st, int first = 0, int count = -1) = 0;
  virtual void flat_step(int first, int n, int n_scenes, int kmax, bool contacts, int n_driven,
                         bool history, bool finish_scenes, hipStream_t st,
                         const FlatWave* waves = nullptr, const int* n_waves = nullptr,
                         int wave_grid = 0, const int* resident_grid = nullptr, bool flat = true) = 0;
  virtual pabd_status set_resident(const std::vector<int>& contact, const std::vector<int>& other,
                                   bool variable, hipStream_t st) = 0;
  // the most bodies a scene run by the resident step kernel may have: those
  // that one pass of the workgroup covers (a contact scene's bodies take four
  // lanes each); larger scenes wait on their partners' loads pass after pass
  // there, and run faster on the flat path, spread over many compute units
  virtual int resident_max(bool contact) const = 0;
  virtual void tile_step(int tile_bodies, const TileTable& tt, int grid, int nsteps,
                         hipStream_t st) = 0;
  virtual void finish_scenes(int n_scenes, hipStream_t st) = 0;
  virtual pabd_status read_bodies(int boff, int n, double* c, double* A, double* v, double* w,
                                  hipStream_t st) = 0;
  virtual pabd_status write_body_field(int body, int field, double value, hipStream_t st) = 0;
  virtual std::string& error() = 0;
  virtual int type_size() const = 0;
  // raw pointers used by the API layer
  virtual SceneDev* scene_table() = 0;
  virtual int* health_ptr() = 0;
  virtual unsigned* polar_ptr() = 0;
  virtual double* rho_ptr() = 0;
  virtual double** history(int* k) = 0;
  virtual pabd_status alloc_history(int K) = 0;
  virtual pabd_status read_contacts(int n, int ccap, std::vector<int>& count,
                                    std::vector<int>& partner,
                                    std::vector<unsigned long long>& key,
                                    std::vector<double>& rec, hipStream_t st) = 0;
  // q^n and velocities of bodies [0, n), the bond-end states of ends [0, ne),
  // the scene table, health bits, last residuals and recorded residual history
  // (saved, or written back)
  virtual pabd_status snapshot(int n, int ne, std::vector<char>& buf, hipStream_t st, bool restore) = 0;
  // flat-path schedule: lanes per contact body, wavefronts per workgroup
  virtual void set_schedule(int contact_lanes, int group_waves) = 0;
  virtual void get_schedule(int* contact_lanes, int* group_waves) const = 0;
  // raw q^n and velocity records of bodies [boff, boff + n) (read, or write back)
  virtual pabd_status raw_bodies(int boff, int n, std::vector<char>& buf, hipStream_t st, bool write) = 0;
  // augmented-bond state of ends [0, ne) as doubles (4 per end)
  virtual pabd_status read_al(int ne, std::vector<double>& out, hipStream_t st) = 0;
  // raw bond-end state records of ends [eoff, eoff + ne) (read, or write back)
  virtual pabd_status raw_al(int eoff, int ne, std::vector<char>& buf, hipStream_t st, bool write) = 0;
  // device memory from `a` instead of the allocator in force, uploads without staging buffers
  virtual void use_memory(const DeviceAllocator& a) = 0;
};

template <typename T>
struct EngineT final : EngineBase {
  Engine<T> e;
  pabd_status allocate(const Caps& c) override { return e.allocate(c); }
  pabd_status upload(const HostScene& hs, int boff, int eoff, int poff, int doff, int sidx,
                     hipStream_t st) override {
    return e.upload(hs, boff, eoff, poff, doff, sidx, st);
  }
  pabd_status clear_bodies(int boff, int n, hipStream_t st, int doff, int nd) override {
    return e.clear_bodies(boff, n, st, doff, nd);
  }
  void factor(hipStream_t st, int first, int count) override { e.launch_factor(st, first, count); }
  void flat_step(int first, int n, int n_scenes, int kmax, bool contacts, int n_driven, bool history,
                 bool fin, hipStream_t st, const FlatWave* waves, const int* n_waves,
                 int wave_grid, const int* resident_grid, bool flat) override {
    (void)first;
    const int saved = e.cap.n;
    e.cap.n = n;  // flat kernels cover bodies [0, n)
    e.launch_flat_step(n_scenes, kmax, contacts, n_driven, history, fin, st, waves, n_waves, wave_grid,
                       resident_grid, flat);
    e.cap.n = saved;
  }
  pabd_status set_resident(const std::vector<int>& contact, const std::vector<int>& other, bool variable,
                           hipStream_t st) override {
    return e.set_resident(contact, other, variable, st);
  }
  int resident_max(bool contact) const override { return contact ? Resident<T>::NT / 4 : Resident<T>::NT; }
  void tile_step(int tb, const TileTable& tt, int grid, int nsteps, hipStream_t st) override {
    View<T> v = e.view();
    switch (tb) {
      case 32:
        hipLaunchKernelGGL((k_tile_step<T, 32, 2>), dim3(grid), dim3(32), 0, st, v, tt, nsteps);
        break;
      case 64:
        hipLaunchKernelGGL((k_tile_step<T, 64, 2>), dim3(grid), dim3(64), 0, st, v, tt, nsteps);
        break;
      case 128:
        hipLaunchKernelGGL((k_tile_step<T, 128, 2>), dim3(grid), dim3(128), 0, st, v, tt, nsteps);
        break;
      default:
        hipLaunchKernelGGL((k_tile_step<T, 256, 2>), dim3(grid), dim3(256), 0, st, v, tt, nsteps);
        break;
    }
  }
  void finish_scenes(int n_scenes, hipStream_t st) override {
    hipLaunchKernelGGL(k_reduce_residual, dim3(std::max(1, n_scenes)), dim3(RED_THREADS), 0, st, e.scenes,
                       n_scenes, (const double*)e.r_num, (const double*)e.r_den, e.rho);
  }
  pabd_status read_bodies(int boff, int n, double* c, double* A, double* v, double* w,
                          hipStream_t st) override {
    constexpr int QR = Rec<T>::Q;
    std::vector<T> q((size_t)QR * n), vl((size_t)VW * n);
    if (n > 0) {
      if (hipMemcpyAsync(q.data(), e.qn + (size_t)QR * boff, q.size() * sizeof(T),
                         hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipMemcpyAsync(vl.data(), e.vel + (size_t)VW * boff, vl.size() * sizeof(T),
                         hipMemcpyDeviceToHost, st) != hipSuccess)
        return fail(PABD_E_DEVICE, "state copy failed");
    }
    if (hipStreamSynchronize(st) != hipSuccess) return fail(PABD_E_DEVICE, "stream sync failed");
    for (int b = 0; b < n; ++b) {
      for (int k = 0; k < 3; ++k) {
        if (c) c[3 * b + k] = (double)q[QR * b + k] + (QR > QW ? (double)q[QR * b + 12 + k] : 0.0);
        if (v) v[3 * b + k] = (double)vl[VW * b + k];
        if (w) w[3 * b + k] = (double)vl[VW * b + 3 + k];
      }
      for (int k = 0; k < 9; ++k)
        if (A) A[9 * b + k] = (double)q[QR * b + 3 + k];
    }
    return PABD_OK;
  }
  pabd_status write_body_field(int body, int field, double value, hipStream_t st) override {
    constexpr int QR = Rec<T>::Q;
    T val = (T)value, zero = (T)0;
    T* dst = field < 12 ? e.qn + (size_t)QR * body + field : e.vel + (size_t)VW * body + (field - 12);
    if (hipMemcpyAsync(dst, &val, sizeof(T), hipMemcpyHostToDevice, st) != hipSuccess)
      return fail(PABD_E_DEVICE, "poke failed");
    if (QR > QW && field < 3 &&  // a poked position has no low part
        hipMemcpyAsync(e.qn + (size_t)QR * body + 12 + field, &zero, sizeof(T), hipMemcpyHostToDevice,
                       st) != hipSuccess)
      return fail(PABD_E_DEVICE, "poke failed");
    if (hipStreamSynchronize(st) != hipSuccess) return fail(PABD_E_DEVICE, "poke failed");
    return PABD_OK;
  }
  std::string& error() override { return e.err; }
  void use_memory(const DeviceAllocator& a) override {
    e.dev = a;
    e.direct_upload = true;
  }
  int type_size() const override { return (int)sizeof(T); }
  SceneDev* scene_table() override { return e.scenes; }
  int* health_ptr() override { return e.health; }
  unsigned* polar_ptr() override { return e.polar; }
  double* rho_ptr() override { return e.rho; }
  double** history(int* k) override {
    *k = e.rh_k;
    return &e.rh_rho;
  }
  pabd_status alloc_history(int K) override {
    if (e.rh_num && e.rh_k >= K) return PABD_OK;
    pabd_status st;
    if ((st = e.alloc(e.rh_num, (size_t)K * e.cap.n)) != PABD_OK) return st;
    if ((st = e.alloc(e.rh_den, (size_t)K * e.cap.n)) != PABD_OK) return st;
    if ((st = e.alloc(e.rh_rho, (size_t)K)) != PABD_OK) return st;
    e.rh_k = K;
    return PABD_OK;
  }
  // contact records of bodies [0, n), each returned as the CW values of the FP64
  // layout (an FP32 record's stiffness is rebuilt from the two bodies' q
  // records and its normal decoded; its friction coefficient reads 0)
  pabd_status read_contacts(int n, int ccap, std::vector<int>& count, std::vector<int>& partner,
                            std::vector<unsigned long long>& key, std::vector<double>& rec,
                            hipStream_t st) override {
    constexpr int W = ContactRec<T>::W, QR = Rec<T>::Q;
    count.assign(n, 0);
    const size_t ns = (size_t)n * ccap;
    partner.assign(ns, 0);
    key.assign(ns, 0);
    std::vector<T> r(W * ns), q;
    if (n > 0 && ccap > 0) {
      if (hipMemcpyAsync(count.data(), e.ccount, n * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipMemcpyAsync(partner.data(), e.ce_partner, ns * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipMemcpyAsync(key.data(), e.ce_key, ns * sizeof(unsigned long long), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipMemcpyAsync(r.data(), e.ce, r.size() * sizeof(T), hipMemcpyDeviceToHost, st) != hipSuccess)
        return fail(PABD_E_DEVICE, "contact copy failed");
      if constexpr (W != CW) {
        q.resize((size_t)QR * n);
        if (hipMemcpyAsync(q.data(), e.qn, q.size() * sizeof(T), hipMemcpyDeviceToHost, st) != hipSuccess)
          return fail(PABD_E_DEVICE, "contact copy failed");
      }
    }
    if (hipStreamSynchronize(st) != hipSuccess) return fail(PABD_E_DEVICE, "stream sync failed");
    rec.assign(CW * ns, 0.0);
    for (size_t k = 0; k < ns; ++k) {
      const T* c = &r[W * k];
      double* o = &rec[CW * k];
      if constexpr (W == CW) {
        for (int d = 0; d < CW; ++d) o[d] = (double)c[d];
      } else {
        const int owner = (int)(k / (size_t)ccap), j = partner[k];
        const T ko = q[(size_t)QR * owner + Q_KAPPA];
        const T kj = j >= 0 && j < n ? q[(size_t)QR * j + Q_KAPPA] : (T)0;
        for (int d = 0; d < 3; ++d) {
          o[d] = (double)c[d];
          o[4 + d] = (double)c[4 + d];
        }
        o[3] = (double)(ko > kj ? ko : kj);
        oct_decode_host((double)c[3], (double)c[7], o + 8);
      }
    }
    return PABD_OK;
  }
  pabd_status read_al(int ne, std::vector<double>& out, hipStream_t st) override {
    std::vector<T> a(4 * (size_t)std::max(ne, 0));
    if (ne > 0 && (hipMemcpyAsync(a.data(), e.al, a.size() * sizeof(T), hipMemcpyDeviceToHost, st) != hipSuccess ||
                   hipStreamSynchronize(st) != hipSuccess))
      return fail(PABD_E_DEVICE, "bond state copy failed");
    out.assign(a.begin(), a.end());
    return PABD_OK;
  }
  pabd_status raw_al(int eoff, int ne, std::vector<char>& buf, hipStream_t st, bool write) override {
    const size_t bytes = (size_t)4 * std::max(ne, 0) * sizeof(T);
    if (!write) buf.resize(bytes);
    if (bytes == 0) return PABD_OK;
    if (buf.size() < bytes) return fail(PABD_E_INVALID, "bond state buffer too small");
    T* d = e.al + (size_t)4 * eoff;
    hipError_t r = write ? hipMemcpyAsync(d, buf.data(), bytes, hipMemcpyHostToDevice, st)
                         : hipMemcpyAsync(buf.data(), d, bytes, hipMemcpyDeviceToHost, st);
    if (r != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
      return fail(PABD_E_DEVICE, "bond state copy failed");
    return PABD_OK;
  }
  pabd_status raw_bodies(int boff, int n, std::vector<char>& buf, hipStream_t st, bool write) override {
    const size_t bq = (size_t)Rec<T>::Q * n * sizeof(T), bv = (size_t)VW * n * sizeof(T);
    T* dq = e.qn + (size_t)Rec<T>::Q * boff;
    T* dv = e.vel + (size_t)VW * boff;
    if (!write) buf.resize(bq + bv);
    if (n <= 0) return PABD_OK;
    hipError_t r1 = write ? hipMemcpyAsync(dq, buf.data(), bq, hipMemcpyHostToDevice, st)
                          : hipMemcpyAsync(buf.data(), dq, bq, hipMemcpyDeviceToHost, st);
    hipError_t r2 = write ? hipMemcpyAsync(dv, buf.data() + bq, bv, hipMemcpyHostToDevice, st)
                          : hipMemcpyAsync(buf.data() + bq, dv, bv, hipMemcpyDeviceToHost, st);
    if (r1 != hipSuccess || r2 != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
      return fail(PABD_E_DEVICE, "body record copy failed");
    return PABD_OK;
  }
  pabd_status snapshot(int n, int ne, std::vector<char>& buf, hipStream_t st, bool restore) override {
    struct Part {
      void* dev;
      size_t bytes;
    };
    const Part parts[] = {{e.qn, (size_t)Rec<T>::Q * n * sizeof(T)},
                          {e.vel, (size_t)VW * n * sizeof(T)},
                          {e.scenes, (size_t)e.cap.s * sizeof(SceneDev)},
                          {e.al, (size_t)4 * std::min(ne, e.cap.e) * sizeof(T)},
                          {e.health, (size_t)e.cap.s * sizeof(int)},
                          {e.rho, (size_t)e.cap.s * sizeof(double)},
                          {e.rh_rho, (size_t)e.rh_k * sizeof(double)}};
    size_t total = 0;
    for (const Part& p : parts) total += p.bytes;
    if (!restore) buf.resize(total);
    if (buf.size() < total) return fail(PABD_E_INVALID, "snapshot buffer too small");
    char* h = buf.data();
    for (const Part& p : parts) {
      if (p.bytes > 0 && p.dev) {
        hipError_t r = restore ? hipMemcpyAsync(p.dev, h, p.bytes, hipMemcpyHostToDevice, st)
                               : hipMemcpyAsync(h, p.dev, p.bytes, hipMemcpyDeviceToHost, st);
        if (r != hipSuccess) return fail(PABD_E_DEVICE, "snapshot copy failed");
      }
      h += p.bytes;
    }
    if (hipStreamSynchronize(st) != hipSuccess) return fail(PABD_E_DEVICE, "snapshot copy failed");
    return PABD_OK;
  }
  void set_schedule(int contact_lanes, int group_waves) override {
    e.contact_lanes = contact_lanes;
    e.group_waves = group_waves;
  }
  void get_schedule(int* contact_lanes, int* group_waves) const override {
    *contact_lanes = e.contact_lanes;
    *group_waves = e.group_waves;
  }
};

std::unique_ptr<EngineBase> make_engine(int precision) {
  if (precision == PABD_FP64) return std::make_unique<EngineT<double>>();
  return std::make_unique<EngineT<float>>();
}

struct Graph {
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  void reset() {
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
    x = nullptr;
    g = nullptr;
  }
  ~Graph() { reset(); }
};

}  // namespace

// ---------------------------------------------------------------------------
// plain scene
// ---------------------------------------------------------------------------

struct pabd_scene {
  HostScene hs;
  std::unique_ptr<EngineBase> eng;
  hipStream_t stream = nullptr;
  int precision = PABD_FP32;
  int debug = 0;
  bool history = false;
  // the whole step in the resident kernel (bodies fit its LDS; not while the
  // residual of every iteration is recorded, which the flat kernels do)
  bool resident = false;
  Graph graph;
  // releases what the handle holds, also after a create that failed part-way
  // (its own stream is drained first; work on callers' streams is the caller's)
  ~pabd_scene() {
    if (stream) (void)hipStreamSynchronize(stream);
    graph.reset();
    eng.reset();
    if (stream) (void)hipStreamDestroy(stream);
  }
};

extern "C" {

const char* pabd_last_error(void) { return g_err.c_str(); }

int32_t pabd_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

size_t pabd_scene_bytes(const pabd_scene_desc* desc) {
  HostScene hs;
  if (!build_host_scene(desc, hs).empty()) return 0;
  return scene_bytes(hs, desc->precision == PABD_FP64 ? 8 : 4);
}

pabd_status pabd_scene_create(const pabd_scene_desc* desc, pabd_scene** out) {
  if (!out) return fail(PABD_E_INVALID, "null output handle");
  *out = nullptr;
  auto s = std::make_unique<pabd_scene>();
  std::string why = build_host_scene(desc, s->hs);
  if (!why.empty()) return fail(PABD_E_INVALID, why);
  if (pabd_device_count() < 1) return fail(PABD_E_DEVICE, "no HIP device");
  s->precision = desc->precision;
  s->eng = make_engine(desc->precision);
  API_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
  Caps c;
  c.n = std::max(1, s->hs.n);
  c.e = std::max(1, s->hs.ne);
  c.s = 1;
  c.p = std::max(1, (int)s->hs.planes.size() / 4);
  c.dr = std::max(1, (int)s->hs.drv_end_i.size());
  c.contacts = s->hs.contact;
  c.cslots = (long long)c.n * s->hs.ccap;
  pabd_status st = s->eng->allocate(c);
  if (st != PABD_OK) return fail(st, s->eng->error());
  s->hs.params.steps_total = INT_MAX;
  s->resident = s->hs.n > 0 && s->hs.n <= s->eng->resident_max(s->hs.contact);
  s->hs.params.resident = s->resident ? 1 : 0;
  st = s->eng->upload(s->hs, 0, 0, 0, 0, 0, s->stream);
  if (st != PABD_OK) return fail(st, s->eng->error());
  if (s->resident) {
    st = s->hs.contact ? s->eng->set_resident({0}, {}, s->hs.variable, s->stream)
                       : s->eng->set_resident({}, {0}, s->hs.variable, s->stream);
    if (st != PABD_OK) return fail(st, s->eng->error());
  }
  s->eng->factor(s->stream);
  API_HIP(hipGetLastError());
  API_HIP(hipStreamSynchronize(s->stream));
  *out = s.release();
  return PABD_OK;
}

pabd_status pabd_scene_destroy(pabd_scene* s) {
  if (!s) return PABD_OK;
  (void)hipDeviceSynchronize();  // steps may have been enqueued on a caller's stream
  delete s;
  return PABD_OK;
}

void* pabd_scene_stream(pabd_scene* s) { return s ? (void*)s->stream : nullptr; }

pabd_status pabd_set_allocator(void* (*alloc)(size_t bytes, void* ctx), void (*release)(void* ptr, void* ctx),
                               void* ctx) {
  if (alloc && !release) return fail(PABD_E_INVALID, "an allocator needs a matching free");
  DeviceAllocator& a = current_allocator();
  a.alloc = alloc;
  a.release = alloc ? release : nullptr;
  a.ctx = alloc ? ctx : nullptr;
  return PABD_OK;
}

static void scene_enqueue_step(pabd_scene* s, hipStream_t st) {
  const HostScene& hs = s->hs;
  if (s->resident && !s->history) {
    const int grid[2] = {hs.contact ? 1 : 0, hs.contact ? 0 : 1};
    s->eng->flat_step(0, std::max(1, hs.n), 1, hs.params.iters, hs.contact, (int)hs.drv_end_i.size(), false,
                      true, st, nullptr, nullptr, 0, grid, false);
    return;
  }
  s->eng->flat_step(0, std::max(1, hs.n), 1, hs.params.iters, hs.contact,
                    (int)hs.drv_end_i.size(), s->history, true, st);
}

pabd_status pabd_scene_step(pabd_scene* s, int32_t nsteps, void* hip_stream) {
  if (!s) return fail(PABD_E_INVALID, "null scene");
  if (nsteps < 0) return fail(PABD_E_INVALID, "negative step count");
  if (nsteps == 0 || s->hs.n == 0) return PABD_OK;
  hipStream_t st = hip_stream ? (hipStream_t)hip_stream : s->stream;
  if (!use_graphs() || s->history) {
    for (int k = 0; k < nsteps; ++k) scene_enqueue_step(s, st);
    API_HIP(hipGetLastError());
    return PABD_OK;
  }
  if (!s->graph.x) {
    hipStream_t cs = s->stream;
    API_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    scene_enqueue_step(s, cs);
    hipError_t e = hipStreamEndCapture(cs, &s->graph.g);
    if (e != hipSuccess) return fail(PABD_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    API_HIP(hipGraphInstantiate(&s->graph.x, s->graph.g, nullptr, nullptr, 0));
  }
  for (int k = 0; k < nsteps; ++k) API_HIP(hipGraphLaunch(s->graph.x, st));
  return PABD_OK;
}

pabd_status pabd_scene_read_state(pabd_scene* s, double* c, double* A, double* v, double* w) {
  if (!s) return fail(PABD_E_INVALID, "null scene");
  API_HIP(hipDeviceSynchronize());
  pabd_status st = s->eng->read_bodies(0, s->hs.n, c, A, v, w, s->stream);
  if (st != PABD_OK) return st;
  int health = 0;
  API_HIP(hipMemcpy(&health, s->eng->health_ptr(), sizeof(int), hipMemcpyDeviceToHost));
  if (health & 1) return fail(PABD_E_DIVERGED, "non-finite state");
  if (health & 2) return fail(PABD_E_DIVERGED, "contact capacity exceeded");
  return PABD_OK;
}

pabd_status pabd_scene_residuals(pabd_scene* s, double* out, int32_t cap, int32_t* k_out) {
  if (!s) return fail(PABD_E_INVALID, "null scene");
  API_HIP(hipDeviceSynchronize());
  const int K = s->hs.params.iters;
  if (k_out) *k_out = K;
  if (!out || cap <= 0) return PABD_OK;
  if (s->history) {
    int kk = 0;
    double** rh = s->eng->history(&kk);
    std::vector<double> h(K, 0.0);
    API_HIP(hipMemcpy(h.data(), *rh, K * sizeof(double), hipMemcpyDeviceToHost));
    for (int k = 0; k < K && k < cap; ++k) out[k] = h[k];
  } else {
    double r = 0.0;
    API_HIP(hipMemcpy(&r, s->eng->rho_ptr(), sizeof(double), hipMemcpyDeviceToHost));
    for (int k = 0; k < K && k < cap; ++k) out[k] = (k == K - 1) ? r : 0.0;
  }
  return PABD_OK;
}

pabd_status pabd_scene_residual(const pabd_scene* s, double* rho_last) {
  if (!s || !rho_last) return fail(PABD_E_INVALID, "null scene or output");
  API_HIP(hipDeviceSynchronize());
  API_HIP(hipMemcpy(rho_last, s->eng->rho_ptr(), sizeof(double), hipMemcpyDeviceToHost));
  return PABD_OK;
}

pabd_status pabd_scene_polar_fallbacks(const pabd_scene* s, int64_t* svd, int64_t* det_nonpositive) {
  if (!s) return fail(PABD_E_INVALID, "null scene");
  API_HIP(hipDeviceSynchronize());
  std::vector<unsigned> c(2 * (size_t)std::max(1, s->hs.n), 0u);
  API_HIP(hipMemcpy(c.data(), s->eng->polar_ptr(), c.size() * sizeof(unsigned), hipMemcpyDeviceToHost));
  int64_t a = 0, d = 0;
  for (size_t k = 0; k < c.size(); k += 2) {
    a += c[k];
    d += c[k + 1];
  }
  if (svd) *svd = a;
  if (det_nonpositive) *det_nonpositive = d;
  return PABD_OK;
}

pabd_status pabd_scene_set_debug(pabd_scene* s, int32_t flags) {
  if (!s) return fail(PABD_E_INVALID, "null scene");
  API_HIP(hipStreamSynchronize(s->stream));
  s->debug = flags;
  s->history = (flags & 2) != 0;
  if (s->history) {
    pabd_status st = s->eng->alloc_history(s->hs.params.iters);
    if (st != PABD_OK) return fail(st, s->eng->error());
  }
  int dbg = flags & 1;
  API_HIP(hipMemcpy((char*)s->eng->scene_table() + offsetof(SceneDev, debug), &dbg, sizeof(int),
                    hipMemcpyHostToDevice));
  // recording every iteration's residual is the flat kernels' work
  const int res = s->resident && !s->history ? 1 : 0;
  API_HIP(hipMemcpy((char*)s->eng->scene_table() + offsetof(SceneDev, resident), &res, sizeof(int),
                    hipMemcpyHostToDevice));
  s->graph.reset();
  return PABD_OK;
}

pabd_status pabd_scene_poke(pabd_scene* s, int32_t body, int32_t field, double value) {
  if (!s) return fail(PABD_E_INVALID, "null scene");
  if (body < 0 || body >= s->hs.n || field < 0 || field > 17) return fail(PABD_E_INVALID, "bad poke target");
  API_HIP(hipDeviceSynchronize());
  return s->eng->write_body_field(body, field, value, s->stream);
}

pabd_status pabd_debug_poke(pabd_scene* s, int32_t body, int32_t field, double value) {
  return pabd_scene_poke(s, body, field, value);
}

pabd_status pabd_scene_bond_state(pabd_scene* s, double* kappa, double* lambda) {
  if (!s) return fail(PABD_E_INVALID, "null scene");
  const int B = (int)s->hs.bond_end.size();
  std::vector<double> al;
  pabd_status st = s->eng->read_al(s->hs.ne, al, s->stream);
  if (st != PABD_OK) return st;
  for (int e = 0; e < B; ++e) {
    const double* a = &al[4 * (size_t)s->hs.bond_end[e]];
    const bool aug = a[3] > 0.0;
    const bool poly = a[3] < 0.0 && a[3] != AL_SLIDER_POINT && a[3] != AL_SLIDER_LINE;
    if (kappa) kappa[e] = aug || poly ? a[0] : s->hs.se[8 * (size_t)s->hs.bond_end[e] + 3];
    if (lambda) lambda[e] = aug ? a[1] : 0.0;
  }
  return PABD_OK;
}

pabd_status pabd_scene_contacts(pabd_scene* s, int32_t cap, int32_t* ci, int32_t* cj,
                                int32_t* feature, double* xi, double* xj, double* normal,
                                double* kappa, int32_t* n_out) {
  if (!s) return fail(PABD_E_INVALID, "null scene");
  if (n_out) *n_out = 0;
  if (!s->hs.contact) return PABD_OK;
  API_HIP(hipDeviceSynchronize());
  std::vector<int> count, partner;
  std::vector<unsigned long long> key;
  std::vector<double> rec;
  pabd_status st = s->eng->read_contacts(s->hs.n, s->hs.ccap, count, partner, key, rec, s->stream);
  if (st != PABD_OK) return st;
  struct C {
    int i, j, f;
    size_t slot;
  };
  std::vector<C> all;
  for (int b = 0; b < s->hs.n; ++b) {
    const int cnt = std::min(count[b], s->hs.ccap);
    for (int k = 0; k < cnt; ++k) {
      const size_t slot = (size_t)b * s->hs.ccap + k;
      if (key[slot] & 1ull) continue;  // j-side copy
      all.push_back({b, partner[slot], (int)((key[slot] >> 1) & 0x7fffffffull), slot});
    }
  }
  std::sort(all.begin(), all.end(), [](const C& a, const C& b) {
    if (a.i != b.i) return a.i < b.i;
    if (a.j != b.j) return a.j < b.j;
    return a.f < b.f;
  });
  for (size_t k = 0; k < all.size() && (int)k < cap; ++k) {
    const double* r = &rec[CW * all[k].slot];
    if (ci) ci[k] = all[k].i;
    if (cj) cj[k] = all[k].j;
    if (feature) feature[k] = all[k].f;
    for (int d = 0; d < 3; ++d) {
      if (xi) xi[3 * k + d] = r[d];
      if (xj) xj[3 * k + d] = r[4 + d];
      if (normal) normal[3 * k + d] = r[8 + d];
    }
    if (kappa) kappa[k] = r[3] / (s->hs.params.h * s->hs.params.h);  // records hold h^2 kappa_c
  }
  if (n_out) *n_out = (int32_t)all.size();
  return PABD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batch
// ---------------------------------------------------------------------------

namespace {

// first-fit allocator of index ranges
struct RangeAlloc {
  std::map<int, int> free_;  // start -> length
  int cap = 0;
  void init(int n) {
    cap = n;
    free_.clear();
    if (n > 0) free_[0] = n;
  }
  int take(int n, int align = 1) {
    if (n <= 0) return 0;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      int s = it->first, len = it->second;
      int a = (s + align - 1) / align * align;
      if (a + n <= s + len) {
        free_.erase(it);
        if (a > s) free_[s] = a - s;
        if (a + n < s + len) free_[a + n] = s + len - (a + n);
        return a;
      }
    }
    return -1;
  }
  void give(int s, int n) {
    if (n <= 0) return;
    auto it = free_.emplace(s, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Slot {
  bool used = false;
  bool tiled = false;
  bool resident = false;  // not tiled, and its whole step runs in the resident kernel
  int boff = 0, n = 0, eoff = 0, ne = 0, poff = 0, np = 0, doff = 0, nd = 0;
  int coff = 0, nslot = 0;  // contact slots [coff, coff + nslot): n bodies x the scene's capacity
  int tile = -1;
  int steps_total = 0;
  long long admitted_at = 0;  // batch substep counter at admission
  size_t bytes = 0;
  int iters = 0;
  bool contact = false;
  std::shared_ptr<HostScene> hs;
};

struct Tile {
  int first = 0, used = 0;
  std::vector<int> slots;
};

}  // namespace

struct pabd_batch {
  int precision = PABD_FP32;
  int max_slots = 0;
  size_t budget = 0, used_bytes = 0;
  Caps caps;
  int n_stream = 0;  // bodies [0, n_stream) are for scenes on the flat path
  std::unique_ptr<EngineBase> eng;
  hipStream_t stream = nullptr;
  std::vector<Slot> slots;
  RangeAlloc stream_bodies, tile_space, ends, planes, driven, cslots;
  std::vector<Tile> tiles;  // index = tile id; used == 0 and no slots: free
  int tile_bodies = 64;
  bool tile_auto = true;
  // flat-path schedule (lanes per contact body, wavefronts per workgroup)
  int contact_lanes = 4, group_waves = 1;
  long long substeps = 0;
  // device tile table
  int *d_first = nullptr, *d_count = nullptr, *d_kmax = nullptr, *d_ntiles = nullptr;
  int tile_table_cap = 0;
  // wave table of the flat-path iterations when contact scenes are on it
  FlatWave* d_waves = nullptr;
  int* d_nwaves = nullptr;
  int wave_table_cap = 0;
  DeviceAllocator dev = current_allocator();
  Graph graph;
  int graph_steps = 0;  // steps one replay of the captured graph advances
  bool dirty = true;
  int grid_tiles = 0;
  bool any_stream = false, any_contact = false;
  int stream_kmax = 0, n_driven_hi = 0;
  int stream_hi = 0;  // one past the highest flat-path body in use
  // launch extents, rounded so that most admissions and releases leave them
  // (and so the captured step graph) unchanged; kernels skip unused slots
  struct Launch {
    int stream_n = 0, driven_n = 0, grid = 0, kmax = 0, tile = 0, wave_grid = 0;
    int res_grid[2] = {0, 0};  // workgroups over the resident lists (contact, other)
    int contact_lanes = 0, group_waves = 0;
    bool stream = false, contact = false, flat = false;
    const int* table = nullptr;
    const FlatWave* waves = nullptr;
    bool operator==(const Launch& o) const {
      return stream_n == o.stream_n && driven_n == o.driven_n && grid == o.grid && kmax == o.kmax &&
             tile == o.tile && stream == o.stream && contact == o.contact && table == o.table &&
             wave_grid == o.wave_grid && waves == o.waves && res_grid[0] == o.res_grid[0] &&
             res_grid[1] == o.res_grid[1] && flat == o.flat && contact_lanes == o.contact_lanes &&
             group_waves == o.group_waves;
    }
  } launch;
  // releases what the handle holds, also after a create that failed part-way
  // (its own stream is drained first; work on callers' streams is the caller's)
  ~pabd_batch() {
    if (stream) (void)hipStreamSynchronize(stream);
    graph.reset();
    dev.put(d_first);
    dev.put(d_count);
    dev.put(d_kmax);
    dev.put(d_waves);
    dev.put(d_nwaves);
    dev.put(d_ntiles);
    eng.reset();
    if (stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

size_t body_cost(int ts) { return (size_t)ts * (4 * (QW + 4) + VW + MW + FW + 4) + 8 * (10 + 8 + 2) + 2 + 4 * 5; }
size_t end_cost(int ts) { return (size_t)ts * EW + 4 + 8 * 4; }
// one contact slot: final and staging copies of the record, partner and key,
// and half a candidate pair
size_t contact_cost(int ts) {
  return (size_t)ts * (ts == 4 ? ContactRec<float>::W : ContactRec<double>::W) + 4 + 8 +
         (ts == 4 ? sizeof(StageRec<float>) : sizeof(StageRec<double>)) + 4;
}
// per flat-path body: broad-phase record, reach, large-list entry, at least 16 candidate pairs
size_t contact_body_cost() { return sizeof(BroadRec) + 8 + 4 + 8 * 16; }

pabd_status batch_tables(pabd_batch* b) {
  // rebuild the device tile table from the host tiles
  std::vector<int> first, count, kmax;
  for (const Tile& t : b->tiles) {
    if (t.slots.empty()) continue;
    int km = 0;
    for (int s : t.slots) km = std::max(km, b->slots[s].iters);
    first.push_back(t.first);
    count.push_back(t.used);
    kmax.push_back(km);
  }
  const int nt = (int)first.size();
  if (nt > b->tile_table_cap) {
    int cap = std::max(nt, 2 * b->tile_table_cap + 16);
    if (b->d_first) {
      API_HIP(hipStreamSynchronize(b->stream));
      b->dev.put(b->d_first);
      b->dev.put(b->d_count);
      b->dev.put(b->d_kmax);
    }
    API_HIP(b->dev.get(reinterpret_cast<void**>(&b->d_first), cap * sizeof(int)));
    API_HIP(b->dev.get(reinterpret_cast<void**>(&b->d_count), cap * sizeof(int)));
    API_HIP(b->dev.get(reinterpret_cast<void**>(&b->d_kmax), cap * sizeof(int)));
    b->tile_table_cap = cap;
  }
  if (!b->d_ntiles) API_HIP(b->dev.get(reinterpret_cast<void**>(&b->d_ntiles), sizeof(int)));
  if (nt) {
    API_HIP(hipMemcpyAsync(b->d_first, first.data(), nt * sizeof(int), hipMemcpyHostToDevice, b->stream));
    API_HIP(hipMemcpyAsync(b->d_count, count.data(), nt * sizeof(int), hipMemcpyHostToDevice, b->stream));
    API_HIP(hipMemcpyAsync(b->d_kmax, kmax.data(), nt * sizeof(int), hipMemcpyHostToDevice, b->stream));
  }
  API_HIP(hipMemcpyAsync(b->d_ntiles, &nt, sizeof(int), hipMemcpyHostToDevice, b->stream));
  API_HIP(hipStreamSynchronize(b->stream));
  b->grid_tiles = nt;
  b->any_stream = false;
  b->any_contact = false;
  b->stream_kmax = 0;
  b->n_driven_hi = 0;
  b->stream_hi = 0;
  bool any_flat = false;  // some scene on the flat path iterates in the flat kernels
  std::vector<int> res_contact, res_other;
  for (int k = 0; k < b->max_slots; ++k) {
    const Slot& s = b->slots[k];
    if (!s.used || s.tiled) continue;
    b->any_stream = true;
    b->any_contact = b->any_contact || s.contact;
    if (s.nd > 0) b->n_driven_hi = std::max(b->n_driven_hi, s.doff + s.nd);
    b->stream_hi = std::max(b->stream_hi, s.boff + std::max(1, s.n));
    if (s.resident) {
      (s.contact ? res_contact : res_other).push_back(k);
    } else {
      any_flat = true;
      b->stream_kmax = std::max(b->stream_kmax, s.iters);
    }
  }
  {
    pabd_status st = b->eng->set_resident(res_contact, res_other, true, b->stream);
    if (st != PABD_OK) return fail(st, b->eng->error());
  }
  auto round_up = [](int x, int q, int cap) { return std::min(cap, (x + q - 1) / q * q); };
  // flat-path waves, when contact scenes share the flat path with others: a
  // contact scene's bodies take contact_lanes lanes each (64 / contact_lanes
  // per wave), any other scene's one lane each (64 per wave); a wave stays
  // within one scene
  b->eng->set_schedule(b->contact_lanes, b->group_waves);
  std::vector<FlatWave> waves;
  if (b->any_contact) {
    std::vector<const Slot*> flat;
    for (const Slot& s : b->slots)
      if (s.used && !s.tiled && !s.resident && s.n > 0) flat.push_back(&s);
    std::sort(flat.begin(), flat.end(), [](const Slot* x, const Slot* y) { return x->boff < y->boff; });
    for (const Slot* s : flat) {
      const int lpb = s->contact ? b->contact_lanes : 1, per = 64 / lpb;
      for (int f = 0; f < s->n; f += per)
        waves.push_back(FlatWave{s->boff + f, std::min(per, s->n - f), lpb, s->contact ? 1 : 0});
    }
  }
  const int nw = (int)waves.size();
  if (b->any_contact) {
    if (nw > b->wave_table_cap || !b->d_waves) {
      const int cap = std::max(nw, 2 * b->wave_table_cap + 256);
      API_HIP(hipStreamSynchronize(b->stream));
      b->dev.put(b->d_waves);
      b->d_waves = nullptr;
      API_HIP(b->dev.get(reinterpret_cast<void**>(&b->d_waves), cap * sizeof(FlatWave)));
      b->wave_table_cap = cap;
    }
    if (!b->d_nwaves) API_HIP(b->dev.get(reinterpret_cast<void**>(&b->d_nwaves), sizeof(int)));
    if (nw)
      API_HIP(hipMemcpyAsync(b->d_waves, waves.data(), nw * sizeof(FlatWave), hipMemcpyHostToDevice, b->stream));
    API_HIP(hipMemcpyAsync(b->d_nwaves, &nw, sizeof(int), hipMemcpyHostToDevice, b->stream));
    API_HIP(hipStreamSynchronize(b->stream));
  }
  pabd_batch::Launch L;
  L.stream = b->any_stream;
  L.contact = b->any_contact;
  L.flat = any_flat;
  L.kmax = b->stream_kmax;
  // rounded like the other extents, so that most admissions reuse the graph
  L.res_grid[0] = res_contact.empty() ? 0 : round_up((int)res_contact.size(), 64, b->max_slots);
  L.res_grid[1] = res_other.empty() ? 0 : round_up((int)res_other.size(), 64, b->max_slots);
  L.stream_n = b->any_stream ? round_up(b->stream_hi, 16384, b->n_stream) : 0;
  L.driven_n = b->n_driven_hi > 0 ? round_up(b->n_driven_hi, 256, b->caps.dr) : 0;
  L.grid = b->grid_tiles > 0 ? round_up(b->grid_tiles, 256, INT_MAX) : 0;
  L.tile = b->tile_bodies;
  L.table = b->d_first;
  // the wave grid is rounded like the other extents, so most admissions and
  // releases reuse the captured graph
  L.wave_grid = b->any_contact ? round_up(std::max(1, nw), 256, INT_MAX) : 0;
  L.waves = b->any_contact ? b->d_waves : nullptr;
  L.contact_lanes = b->contact_lanes;
  L.group_waves = b->group_waves;
  if (!(L == b->launch)) {
    b->launch = L;
    b->graph.reset();
  }
  return PABD_OK;
}

// nsteps steps of every resident scene: the flat path one step after another,
// the tiles in one launch that runs all nsteps
void batch_enqueue(pabd_batch* b, int nsteps, hipStream_t st) {
  const pabd_batch::Launch& L = b->launch;
  if (L.grid > 0) {
    TileTable tt{b->d_first, b->d_count, b->d_kmax, b->d_ntiles};
    b->eng->tile_step(L.tile, tt, L.grid, nsteps, st);
  }
  if (L.stream) {
    for (int k = 0; k < nsteps; ++k) {
      b->eng->flat_step(0, L.stream_n, b->max_slots, L.kmax, L.contact, L.driven_n, false, false, st,
                        L.wave_grid > 0 ? b->d_waves : nullptr, b->d_nwaves, L.wave_grid, L.res_grid, L.flat);
      // scenes on the flat path: residual reduction and step counters (tiled
      // and resident scenes do both inside their kernels)
      if (L.flat) b->eng->finish_scenes(b->max_slots, st);
    }
  }
}

pabd_status place_tiled(pabd_batch* b, int slot, int n) {
  Slot& s = b->slots[slot];
  for (size_t t = 0; t < b->tiles.size(); ++t) {
    Tile& T = b->tiles[t];
    if (!T.slots.empty() && T.used + n <= b->tile_bodies) {
      s.tile = (int)t;
      s.boff = T.first + T.used;
      T.used += n;
      T.slots.push_back(slot);
      return PABD_OK;
    }
  }
  int first = b->tile_space.take(b->tile_bodies, b->tile_bodies);
  if (first < 0) return PABD_E_BUSY;
  int tid = -1;
  for (size_t t = 0; t < b->tiles.size(); ++t)
    if (b->tiles[t].slots.empty() && b->tiles[t].used == 0 && b->tiles[t].first < 0) {
      tid = (int)t;
      break;
    }
  if (tid < 0) {
    tid = (int)b->tiles.size();
    b->tiles.push_back(Tile{});
  }
  Tile& T = b->tiles[tid];
  T.first = first;
  T.used = n;
  T.slots = {slot};
  s.tile = tid;
  s.boff = first;
  return PABD_OK;
}

void unplace_tiled(pabd_batch* b, int slot) {
  Slot& s = b->slots[slot];
  Tile& T = b->tiles[s.tile];
  T.slots.erase(std::find(T.slots.begin(), T.slots.end(), slot));
  if (T.slots.empty()) {
    b->tile_space.give(T.first, b->tile_bodies);
    T.first = -1;
    T.used = 0;
  } else {
    int hi = 0;
    for (int o : T.slots) hi = std::max(hi, b->slots[o].boff + b->slots[o].n - T.first);
    T.used = hi;
  }
  s.tile = -1;
}

pabd_status batch_place_and_upload(pabd_batch* b, int slot) {
  Slot& s = b->slots[slot];
  const HostScene& hs = *s.hs;
  const bool tiled = !hs.contact && !hs.driven && !hs.variable && hs.n > 0 && hs.n <= b->tile_bodies;
  s.tiled = tiled;
  // In a batch the flat path's scenes stay in the flat kernels: a resident
  // workgroup holds a whole compute unit for one scene's step, which beside
  // the flat kernels' other scenes costs more than it saves (served mix, all
  // requests queued: 2.96e9 body-iterations/s with resident scenes against
  // 3.22e9 without); a single scene alone gains from it (pabd_scene_step).
  s.resident = false;
  if (tiled) {
    pabd_status st = place_tiled(b, slot, hs.n);
    if (st != PABD_OK) return st;
  } else {
    s.boff = b->stream_bodies.take(std::max(1, hs.n));
    if (s.boff < 0) return PABD_E_BUSY;
  }
  s.eoff = b->ends.take(std::max(1, hs.ne));
  // planes and driven bonds take table space only when the scene has them
  s.np = (int)hs.planes.size() / 4;
  s.poff = s.np > 0 ? b->planes.take(s.np) : 0;
  s.nd = (int)hs.drv_end_i.size();
  s.doff = s.nd > 0 ? b->driven.take(s.nd) : 0;
  // contact slots: the scene's own capacity per body, from the batch's pool
  s.nslot = hs.contact ? hs.n * hs.ccap : 0;
  s.coff = s.nslot > 0 ? b->cslots.take(s.nslot) : 0;
  auto undo = [&]() {
    if (s.tiled) unplace_tiled(b, slot);
    else if (s.boff >= 0) b->stream_bodies.give(s.boff, std::max(1, hs.n));
    if (s.eoff >= 0) b->ends.give(s.eoff, std::max(1, hs.ne));
    if (s.np > 0 && s.poff >= 0) b->planes.give(s.poff, s.np);
    if (s.nd > 0 && s.doff >= 0) b->driven.give(s.doff, s.nd);
    if (s.nslot > 0 && s.coff >= 0) b->cslots.give(s.coff, s.nslot);
  };
  if (s.eoff < 0 || s.poff < 0 || s.doff < 0 || s.coff < 0) {
    undo();
    return PABD_E_BUSY;
  }
  HostScene copy = hs;
  copy.params.steps_total = s.steps_total;
  copy.params.ccap = hs.ccap;
  copy.params.ce_off = s.coff;
  copy.params.tiled = tiled ? 1 : 0;
  copy.params.resident = s.resident ? 1 : 0;
  pabd_status st = b->eng->upload(copy, s.boff, s.eoff, s.poff, s.doff, slot, b->stream);
  if (st != PABD_OK) {
    undo();
    return fail(st, b->eng->error());
  }
  b->eng->factor(b->stream, s.boff, hs.n);
  API_HIP(hipGetLastError());
  API_HIP(hipStreamSynchronize(b->stream));
  return PABD_OK;
}

}  // namespace

extern "C" {

pabd_status pabd_batch_create(int32_t max_slots, size_t hbm_budget, int32_t precision,
                              pabd_batch** out) {
  if (!out) return fail(PABD_E_INVALID, "null output handle");
  *out = nullptr;
  if (max_slots < 1) return fail(PABD_E_INVALID, "max_slots must be >= 1");
  if (precision != PABD_FP32 && precision != PABD_FP64) return fail(PABD_E_INVALID, "unknown precision");
  if (pabd_device_count() < 1) return fail(PABD_E_DEVICE, "no HIP device");
  auto b = std::make_unique<pabd_batch>();
  b->precision = precision;
  b->max_slots = max_slots;
  b->budget = hbm_budget;
  const int ts = precision == PABD_FP64 ? 8 : 4;
  // capacity: each pool -- bodies on the flat path, tiled bodies, bond ends,
  // contact slots -- holds a whole budget's worth of its own item (at most 2^28
  // items), so that every scene whose pabd_scene_bytes fits the budget fits an
  // empty batch; the device memory is then at most about four budgets, while
  // admission keeps the resident scenes' bytes within one
  // (scaled down together when that would exceed 85 % of the device's free memory)
  const size_t lim = (size_t)1 << 28;
  const size_t fb = body_cost(ts) + contact_body_cost();
  size_t n_stream = std::min(lim, std::max<size_t>(1024, hbm_budget / fb));
  size_t n_tiled = std::min(lim, std::max<size_t>(1024, hbm_budget / body_cost(ts)));
  size_t n_ends = std::min(lim, std::max<size_t>(4096, hbm_budget / end_cost(ts)));
  size_t n_slots = std::min(lim, std::max<size_t>(65536, hbm_budget / contact_cost(ts)));
  {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) {
      const double want = (double)n_stream * fb + (double)n_tiled * body_cost(ts) +
                          (double)n_ends * end_cost(ts) + (double)n_slots * contact_cost(ts);
      const double room = 0.85 * (double)free_b;
      if (want > room) {
        const double f = room / want;
        n_stream = std::max<size_t>(1024, (size_t)(n_stream * f));
        n_tiled = std::max<size_t>(1024, (size_t)(n_tiled * f));
        n_ends = std::max<size_t>(4096, (size_t)(n_ends * f));
        n_slots = std::max<size_t>(65536, (size_t)(n_slots * f));
      }
    } else {
      (void)hipGetLastError();
    }
  }
  n_tiled = (n_tiled + 255) / 256 * 256;
  b->n_stream = (int)n_stream;
  b->caps.n = (int)(n_stream + n_tiled);
  b->caps.e = (int)n_ends;
  b->caps.s = max_slots;
  b->caps.p = 4 * max_slots + 16;
  b->caps.dr = std::max(64, (int)(n_stream / 4));
  b->caps.contacts = true;
  b->caps.cslots = (long long)n_slots;
  b->caps.nc = (int)n_stream;  // contacts only on the flat path
  b->eng = make_engine(precision);
  API_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
  pabd_status st = b->eng->allocate(b->caps);
  if (st != PABD_OK) return fail(st, b->eng->error());
  // scene table entries start inactive (no bodies, zero steps)
  std::vector<SceneDev> sc(max_slots);
  for (auto& s : sc) {
    s = SceneDev{};
    s.h = 1.0;
    s.iters = 1;
    s.cell = 1.0;
  }
  API_HIP(hipMemcpy(b->eng->scene_table(), sc.data(), sc.size() * sizeof(SceneDev), hipMemcpyHostToDevice));
  b->slots.resize(max_slots);
  b->stream_bodies.init(b->n_stream);
  b->tile_space.init(b->caps.n);
  b->tile_space.take(b->n_stream);  // tile space begins after the flat-path bodies
  {
    // re-init tile space as [n_stream, n)
    b->tile_space.init(0);
    b->tile_space.cap = b->caps.n;
    b->tile_space.free_.clear();
    b->tile_space.free_[b->n_stream] = b->caps.n - b->n_stream;
  }
  b->ends.init(b->caps.e);
  b->planes.init(b->caps.p);
  b->driven.init(b->caps.dr);
  b->cslots.init((int)b->caps.cslots);
  *out = b.release();
  return PABD_OK;
}

pabd_status pabd_batch_destroy(pabd_batch* b) {
  if (!b) return PABD_OK;
  (void)hipDeviceSynchronize();  // steps may have been enqueued on a caller's stream
  delete b;
  return PABD_OK;
}

void* pabd_batch_stream(pabd_batch* b) { return b ? (void*)b->stream : nullptr; }

pabd_status pabd_batch_sync(pabd_batch* b) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  API_HIP(hipStreamSynchronize(b->stream));
  return PABD_OK;
}

pabd_status pabd_batch_memory(pabd_batch* b, size_t* used, size_t* budget) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  if (used) *used = b->used_bytes;
  if (budget) *budget = b->budget;
  return PABD_OK;
}

pabd_status pabd_batch_admit(pabd_batch* b, const pabd_scene_desc* desc, int32_t nsteps,
                             int32_t* slot_out) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  if (nsteps < 0) return fail(PABD_E_INVALID, "negative step count");
  if (!desc || desc->precision != b->precision)
    return fail(PABD_E_INVALID, "scene precision differs from the batch precision");
  auto hs = std::make_shared<HostScene>();
  std::string why = build_host_scene(desc, *hs);
  if (!why.empty()) return fail(PABD_E_INVALID, why);
  if (hs->contact && (long long)hs->n * hs->ccap > b->caps.cslots)
    return fail(PABD_E_INVALID, "the scene needs more contact slots (bodies x max_contacts_per_body) than the batch holds");
  const size_t bytes = scene_bytes(*hs, b->precision == PABD_FP64 ? 8 : 4);
  if (b->used_bytes + bytes > b->budget) return fail(PABD_E_BUSY, "HBM budget exhausted");
  int slot = -1;
  for (int k = 0; k < b->max_slots; ++k)
    if (!b->slots[k].used) {
      slot = k;
      break;
    }
  if (slot < 0) return fail(PABD_E_BUSY, "no free slot");
  // the flat path is not yet recorded in a graph: finish in-flight work first
  API_HIP(hipStreamSynchronize(b->stream));
  Slot& s = b->slots[slot];
  s = Slot{};
  s.hs = hs;
  s.n = hs->n;
  s.ne = hs->ne;
  s.iters = hs->params.iters;
  s.contact = hs->contact;
  s.steps_total = nsteps;
  s.admitted_at = b->substeps;
  s.bytes = bytes;
  pabd_status st = batch_place_and_upload(b, slot);
  if (st != PABD_OK) {
    s = Slot{};
    return st == PABD_E_BUSY ? fail(st, "no contiguous room for the scene") : st;
  }
  s.used = true;
  b->used_bytes += bytes;
  b->dirty = true;
  if (slot_out) *slot_out = slot;
  return PABD_OK;
}

pabd_status pabd_batch_release(pabd_batch* b, int32_t slot) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  if (slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(PABD_E_NOTFOUND, "slot not in use");
  API_HIP(hipStreamSynchronize(b->stream));
  Slot& s = b->slots[slot];
  pabd_status st = b->eng->clear_bodies(s.boff, std::max(1, s.n), b->stream, s.doff, s.nd);
  if (st != PABD_OK) return fail(st, b->eng->error());
  SceneDev off{};
  off.h = 1.0;
  off.iters = 1;
  off.cell = 1.0;
  API_HIP(hipMemcpy(b->eng->scene_table() + slot, &off, sizeof(SceneDev), hipMemcpyHostToDevice));
  if (s.tiled) unplace_tiled(b, slot);
  else b->stream_bodies.give(s.boff, std::max(1, s.n));
  b->ends.give(s.eoff, std::max(1, s.ne));
  if (s.np > 0) b->planes.give(s.poff, s.np);
  if (s.nd > 0) b->driven.give(s.doff, s.nd);
  if (s.nslot > 0) b->cslots.give(s.coff, s.nslot);
  b->used_bytes -= s.bytes;
  s = Slot{};
  b->dirty = true;
  return PABD_OK;
}

pabd_status pabd_batch_steps(pabd_batch* b, int32_t nsteps, void* hip_stream) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  if (nsteps < 1 || nsteps > PABD_MAX_STEPS_PER_LAUNCH) return fail(PABD_E_INVALID, "nsteps out of range");
  hipStream_t st = hip_stream ? (hipStream_t)hip_stream : b->stream;
  if (b->dirty) {  // new tables; the graph is rebuilt only if the launch extents changed
    pabd_status s2 = batch_tables(b);
    if (s2 != PABD_OK) return s2;
    b->dirty = false;
  }
  if (use_graphs()) {
    if (b->graph.x && b->graph_steps != nsteps) b->graph.reset();
    if (!b->graph.x) {
      API_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      batch_enqueue(b, nsteps, b->stream);
      hipError_t e = hipStreamEndCapture(b->stream, &b->graph.g);
      if (e != hipSuccess) return fail(PABD_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
      API_HIP(hipGraphInstantiate(&b->graph.x, b->graph.g, nullptr, nullptr, 0));
      b->graph_steps = nsteps;
    }
    API_HIP(hipGraphLaunch(b->graph.x, st));
  } else {
    batch_enqueue(b, nsteps, st);
    API_HIP(hipGetLastError());
  }
  b->substeps += nsteps;
  return PABD_OK;
}

pabd_status pabd_batch_step(pabd_batch* b, void* hip_stream) { return pabd_batch_steps(b, 1, hip_stream); }

pabd_status pabd_batch_steps_done(pabd_batch* b, int32_t slot, int32_t* steps) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  if (slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(PABD_E_NOTFOUND, "slot not in use");
  const Slot& s = b->slots[slot];
  long long d = b->substeps - s.admitted_at;
  if (steps) *steps = (int32_t)std::min<long long>(d, s.steps_total);
  return PABD_OK;
}

pabd_status pabd_batch_poll(pabd_batch* b, int32_t* done, int32_t cap, int32_t* n_done) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  int n = 0;
  for (int k = 0; k < b->max_slots; ++k) {
    const Slot& s = b->slots[k];
    if (!s.used) continue;
    if (b->substeps - s.admitted_at >= s.steps_total) {
      if (done && n < cap) done[n] = k;
      ++n;
    }
  }
  if (n_done) *n_done = n;
  return PABD_OK;
}

pabd_status pabd_batch_read_state(pabd_batch* b, int32_t slot, double* c, double* A, double* v,
                                  double* w) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  if (slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(PABD_E_NOTFOUND, "slot not in use");
  API_HIP(hipDeviceSynchronize());
  const Slot& s = b->slots[slot];
  pabd_status st = b->eng->read_bodies(s.boff, s.n, c, A, v, w, b->stream);
  if (st != PABD_OK) return st;
  int health = 0;
  API_HIP(hipMemcpy(&health, b->eng->health_ptr() + slot, sizeof(int), hipMemcpyDeviceToHost));
  if (health & 1) return fail(PABD_E_DIVERGED, "non-finite state");
  if (health & 2) return fail(PABD_E_DIVERGED, "contact capacity exceeded");
  return PABD_OK;
}

pabd_status pabd_batch_residual(pabd_batch* b, int32_t slot, double* rho_last) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  if (slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(PABD_E_NOTFOUND, "slot not in use");
  API_HIP(hipDeviceSynchronize());
  API_HIP(hipMemcpy(rho_last, b->eng->rho_ptr() + slot, sizeof(double), hipMemcpyDeviceToHost));
  return PABD_OK;
}

pabd_status pabd_batch_faults(pabd_batch* b, int32_t* slots, int32_t* codes, int32_t cap, int32_t* n_out) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  API_HIP(hipDeviceSynchronize());
  std::vector<int> h(b->max_slots, 0);
  API_HIP(hipMemcpy(h.data(), b->eng->health_ptr(), h.size() * sizeof(int), hipMemcpyDeviceToHost));
  int n = 0;
  for (int k = 0; k < b->max_slots; ++k) {
    if (!b->slots[k].used || h[k] == 0) continue;
    if (n < cap) {
      if (slots) slots[n] = k;
      if (codes) codes[n] = h[k];
    }
    ++n;
  }
  if (n_out) *n_out = n;
  return PABD_OK;
}

pabd_status pabd_batch_poke(pabd_batch* b, int32_t slot, int32_t body, int32_t field, double value) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  if (slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(PABD_E_NOTFOUND, "slot not in use");
  const Slot& s = b->slots[slot];
  if (body < 0 || body >= s.n || field < 0 || field > 17) return fail(PABD_E_INVALID, "bad poke target");
  API_HIP(hipDeviceSynchronize());
  return b->eng->write_body_field(s.boff + body, field, value, b->stream);
}

pabd_status pabd_batch_polar_fallbacks(pabd_batch* b, int32_t slot, int64_t* svd, int64_t* det_nonpositive) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  if (slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(PABD_E_NOTFOUND, "slot not in use");
  API_HIP(hipDeviceSynchronize());
  const Slot& s = b->slots[slot];
  std::vector<unsigned> c(2 * (size_t)std::max(1, s.n), 0u);
  API_HIP(hipMemcpy(c.data(), b->eng->polar_ptr() + 2 * (size_t)s.boff, c.size() * sizeof(unsigned),
                    hipMemcpyDeviceToHost));
  int64_t a = 0, d = 0;
  for (size_t k = 0; k < c.size(); k += 2) {
    a += c[k];
    d += c[k + 1];
  }
  if (svd) *svd = a;
  if (det_nonpositive) *det_nonpositive = d;
  return PABD_OK;
}

// one past the highest body and the highest bond end any resident scene uses:
// the extent of a snapshot of the batch's state
static void batch_extent(const pabd_batch* b, int* n, int* ne) {
  int hn = 0, he = 0;
  for (const Slot& s : b->slots) {
    if (!s.used) continue;
    hn = std::max(hn, s.boff + std::max(1, s.n));
    he = std::max(he, s.eoff + std::max(1, s.ne));
  }
  *n = std::min(hn, b->caps.n);
  *ne = std::min(he, b->caps.e);
}

static pabd_status batch_repack(pabd_batch* b, int tile_bodies) {
  // read back every resident scene's state, re-place all scenes with the new
  // tile size, and upload again
  API_HIP(hipDeviceSynchronize());
  std::vector<int> live;
  for (int k = 0; k < b->max_slots; ++k)
    if (b->slots[k].used) live.push_back(k);
  std::vector<int> sc_steps(b->max_slots, 0);
  {
    std::vector<SceneDev> tab(b->max_slots);
    API_HIP(hipMemcpy(tab.data(), b->eng->scene_table(), tab.size() * sizeof(SceneDev), hipMemcpyDeviceToHost));
    for (int k : live) sc_steps[k] = tab[k].step;
  }
  // the device records move bit for bit (an FP32 position is a (hi, lo) pair that
  // a round trip through FP64 need not reproduce)
  // The bond-end states (augmented multipliers and stiffnesses) move the same
  // way: an upload would restart them from the descriptor.
  std::vector<std::vector<char>> raw(b->max_slots), raw_ends(b->max_slots);
  for (int k : live) {
    Slot& s = b->slots[k];
    pabd_status st = b->eng->raw_bodies(s.boff, s.n, raw[k], b->stream, false);
    if (st != PABD_OK) return st;
    if ((st = b->eng->raw_al(s.eoff, s.ne, raw_ends[k], b->stream, false)) != PABD_OK) return st;
  }
  for (int k : live) {
    Slot& s = b->slots[k];
    HostScene& hs = *s.hs;
    std::vector<double> c(3 * s.n), A(9 * s.n), v(3 * s.n), w(3 * s.n);
    pabd_status st = b->eng->read_bodies(s.boff, s.n, c.data(), A.data(), v.data(), w.data(), b->stream);
    if (st != PABD_OK) return st;
    auto fresh = std::make_shared<HostScene>(hs);
    for (int i = 0; i < s.n; ++i) {
      for (int d = 0; d < 3; ++d) fresh->qn[12 * i + d] = c[3 * i + d];
      for (int d = 0; d < 9; ++d) fresh->qn[12 * i + 3 + d] = A[9 * i + d];
      for (int d = 0; d < 3; ++d) {
        fresh->vel[8 * i + d] = v[3 * i + d];
        fresh->vel[8 * i + 3 + d] = w[3 * i + d];
      }
    }
    s.hs = fresh;
  }
  for (int k : live) {
    Slot& s = b->slots[k];
    pabd_status st = b->eng->clear_bodies(s.boff, std::max(1, s.n), b->stream, s.doff, s.nd);
    if (st != PABD_OK) return fail(st, b->eng->error());
    if (s.tiled) unplace_tiled(b, k);
    else b->stream_bodies.give(s.boff, std::max(1, s.n));
    b->ends.give(s.eoff, std::max(1, s.ne));
    if (s.np > 0) b->planes.give(s.poff, s.np);
    if (s.nd > 0) b->driven.give(s.doff, s.nd);
    if (s.nslot > 0) b->cslots.give(s.coff, s.nslot);
  }
  b->tiles.clear();
  b->tile_bodies = tile_bodies;
  for (int k : live) {
    Slot& s = b->slots[k];
    pabd_status st = batch_place_and_upload(b, k);
    if (st != PABD_OK) return fail(PABD_E_OOM, "repack did not fit");
    // restore the scene's records, bond-end states and step counter
    st = b->eng->raw_bodies(s.boff, s.n, raw[k], b->stream, true);
    if (st != PABD_OK) return st;
    if ((st = b->eng->raw_al(s.eoff, s.ne, raw_ends[k], b->stream, true)) != PABD_OK) return st;
    SceneDev* d = b->eng->scene_table() + k;
    API_HIP(hipMemcpy((char*)d + offsetof(SceneDev, step), &sc_steps[k], sizeof(int), hipMemcpyHostToDevice));
  }
  b->eng->factor(b->stream);
  API_HIP(hipStreamSynchronize(b->stream));
  b->dirty = true;
  return PABD_OK;
}

pabd_status pabd_batch_time_tile_kernel(pabd_batch* b, int32_t reps, int32_t nsteps, double* avg_ms) {
  if (!b || reps < 1 || !avg_ms) return fail(PABD_E_INVALID, "bad arguments");
  if (nsteps < 1 || nsteps > PABD_MAX_STEPS_PER_LAUNCH) return fail(PABD_E_INVALID, "nsteps out of range");
  *avg_ms = 0.0;
  if (b->dirty) {
    pabd_status s2 = batch_tables(b);
    if (s2 != PABD_OK) return s2;
    b->dirty = false;
  }
  if (b->grid_tiles == 0) return PABD_OK;
  struct Events {  // released on every path, failures included
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } ev;
  API_HIP(hipEventCreate(&ev.e0));
  API_HIP(hipEventCreate(&ev.e1));
  TileTable tt{b->d_first, b->d_count, b->d_kmax, b->d_ntiles};
  b->eng->tile_step(b->tile_bodies, tt, b->grid_tiles, nsteps, b->stream);  // warm
  API_HIP(hipEventRecord(ev.e0, b->stream));
  for (int r = 0; r < reps; ++r) b->eng->tile_step(b->tile_bodies, tt, b->grid_tiles, nsteps, b->stream);
  API_HIP(hipEventRecord(ev.e1, b->stream));
  API_HIP(hipEventSynchronize(ev.e1));
  float ms = 0.f;
  API_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
  *avg_ms = (double)ms / reps;
  return PABD_OK;
}

pabd_status pabd_batch_layout(pabd_batch* b, int32_t* n_bodies, int32_t* n_tiles, int32_t* tile_bodies) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  int nb = 0, nt = 0;
  for (const Slot& s : b->slots)
    if (s.used) nb += s.n;
  for (const Tile& t : b->tiles)
    if (!t.slots.empty()) ++nt;
  if (n_bodies) *n_bodies = nb;
  if (n_tiles) *n_tiles = nt;
  if (tile_bodies) *tile_bodies = b->tile_bodies;
  return PABD_OK;
}

pabd_status pabd_batch_set_tile(pabd_batch* b, int32_t tile_bodies) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  if (tile_bodies == 0) {
    b->tile_auto = true;
    return PABD_OK;
  }
  if (tile_bodies != 32 && tile_bodies != 64 && tile_bodies != 128 && tile_bodies != 256)
    return fail(PABD_E_INVALID, "tile size must be 32, 64, 128 or 256");
  b->tile_auto = false;
  if (tile_bodies == b->tile_bodies) return PABD_OK;
  return batch_repack(b, tile_bodies);
}

pabd_status pabd_batch_autotune(pabd_batch* b, int32_t* tile_out) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  // candidates: tile sizes that hold the largest tiled scene
  int largest = 0;
  for (const Slot& s : b->slots)
    if (s.used && !s.hs->contact && !s.hs->driven && !s.hs->variable) largest = std::max(largest, s.n);
  std::vector<int> cand;
  for (int t : {32, 64, 128, 256})
    if (t >= largest) cand.push_back(t);
  if (cand.empty()) cand.push_back(256);
  API_HIP(hipDeviceSynchronize());
  std::vector<char> snap;
  pabd_status st;
  double best_t = 1e300;
  int best = b->tile_bodies;
  long long substeps0 = b->substeps;
  // Every candidate holds every tiled scene, so the flat-path work is the same
  // for all of them and only the tile kernel is timed: with HIP events, at the
  // steps per launch the batch last ran (10 before any), best of three rounds,
  // each from the saved state so that no scene's step budget runs out midway.
  const int ns = b->graph_steps > 0 ? b->graph_steps : 10;
  for (int t : cand) {
    if (t != b->tile_bodies && (st = batch_repack(b, t)) != PABD_OK) return st;
    int n = 0, ne = 0;  // the state of the scenes as now placed
    batch_extent(b, &n, &ne);
    if ((st = b->eng->snapshot(n, ne, snap, b->stream, false)) != PABD_OK) return st;
    double dt = 1e300;
    for (int round = 0; round < 3; ++round) {
      double ms = 0.0;
      if ((st = pabd_batch_time_tile_kernel(b, 1, ns, &ms)) != PABD_OK) return st;
      if ((st = b->eng->snapshot(n, ne, snap, b->stream, true)) != PABD_OK) return st;
      dt = std::min(dt, ms);
    }
    b->substeps = substeps0;
    if (dt < best_t) {
      best_t = dt;
      best = t;
    }
  }
  if (best != b->tile_bodies && (st = batch_repack(b, best)) != PABD_OK) return st;
  b->tile_auto = false;
  if (tile_out) *tile_out = best;
  return PABD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// launch schedules and the tuner
// ---------------------------------------------------------------------------

namespace {

// cache key of a tuned schedule: device architecture, precision, kind (0 batch,
// 1 plain scene) and size buckets (bit lengths of counts)
struct TuneKey {
  std::string arch;
  int precision = 0, kind = 0;
  int bucket[5] = {0, 0, 0, 0, 0};
  bool operator<(const TuneKey& o) const {
    if (arch != o.arch) return arch < o.arch;
    if (precision != o.precision) return precision < o.precision;
    if (kind != o.kind) return kind < o.kind;
    return std::lexicographical_compare(bucket, bucket + 5, o.bucket, o.bucket + 5);
  }
};

std::mutex g_tune_mu;
std::map<TuneKey, pabd_schedule>& tune_cache() {
  static std::map<TuneKey, pabd_schedule> m;
  return m;
}

int bit_length(long long x) {
  int b = 0;
  for (; x > 0; x >>= 1) ++b;
  return b;
}

std::string device_arch() {
  int d = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&d) != hipSuccess || hipGetDeviceProperties(&p, d) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  return p.gcnArchName;
}

bool valid_lanes(int l) { return l == 1 || l == 2 || l == 4 || l == 8 || l == 16; }
bool valid_waves(int g) { return g == 1 || g == 2 || g == 4; }

const int kLaneCandidates[] = {1, 2, 4, 8, 16};
const int kWaveCandidates[] = {1, 2, 4};

struct EventPair {  // released on every path, failures included
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~EventPair() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// Average duration in ms of one step, timed with HIP events on `st` over
// `reps` calls of step() after one untimed call (which may capture a graph).
template <typename Step>
pabd_status time_steps(hipStream_t st, int reps, Step step, double* ms_out) {
  EventPair ev;
  API_HIP(hipEventCreate(&ev.e0));
  API_HIP(hipEventCreate(&ev.e1));
  pabd_status s = step();
  if (s != PABD_OK) return s;
  API_HIP(hipEventRecord(ev.e0, st));
  for (int r = 0; r < reps; ++r)
    if ((s = step()) != PABD_OK) return s;
  API_HIP(hipEventRecord(ev.e1, st));
  API_HIP(hipEventSynchronize(ev.e1));
  float ms = 0.f;
  API_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
  *ms_out = (double)ms / reps;
  return PABD_OK;
}

// A candidate replaces the schedule in force only when it is faster by more
// than this fraction (timing noise between candidates is a few per cent).
constexpr double kTuneMargin = 0.03;

// Coordinate search over the flat-path schedule: contact lanes (when `lanes`),
// then wavefronts per workgroup, each candidate applied by apply(cl, gw) and
// timed by timed(&ms) (best of three rounds, each from the saved state, which
// restore() writes back).  Leaves the best schedule in *cl, *gw.
template <typename Apply, typename Timed, typename Restore>
pabd_status search_flat(bool lanes, int* cl, int* gw, Apply apply, Timed timed, Restore restore) {
  auto best_of = [&](int c, int g, double* out) -> pabd_status {
    apply(c, g);
    double best = 1e300;
    for (int round = 0; round < 3; ++round) {
      double ms = 0.0;
      pabd_status s = timed(&ms);
      if (s != PABD_OK) return s;
      if ((s = restore()) != PABD_OK) return s;
      best = std::min(best, ms);
    }
    *out = best;
    return PABD_OK;
  };
  pabd_status s;
  if (lanes) {
    double best_t = 0.0;
    if ((s = best_of(*cl, *gw, &best_t)) != PABD_OK) return s;
    int best = *cl;
    for (int c : kLaneCandidates) {
      if (c == *cl) continue;
      double t = 0.0;
      if ((s = best_of(c, *gw, &t)) != PABD_OK) return s;
      if (t < (1.0 - kTuneMargin) * best_t) {
        best_t = t;
        best = c;
      }
    }
    *cl = best;
  }
  double best_t = 0.0;
  if ((s = best_of(*cl, *gw, &best_t)) != PABD_OK) return s;
  int best = *gw;
  for (int g : kWaveCandidates) {
    if (g == *gw) continue;
    double t = 0.0;
    if ((s = best_of(*cl, g, &t)) != PABD_OK) return s;
    if (t < (1.0 - kTuneMargin) * best_t) {
      best_t = t;
      best = g;
    }
  }
  *gw = best;
  apply(*cl, *gw);
  return PABD_OK;
}

}  // namespace

extern "C" {

void pabd_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_cache().clear();
}

int32_t pabd_tune_cache_size(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return (int32_t)tune_cache().size();
}

pabd_status pabd_batch_get_schedule(const pabd_batch* b, pabd_schedule* out) {
  if (!b || !out) return fail(PABD_E_INVALID, "null argument");
  out->tile_bodies = b->tile_bodies;
  out->contact_lanes = b->contact_lanes;
  out->group_waves = b->group_waves;
  out->from_cache = 0;
  return PABD_OK;
}

pabd_status pabd_batch_set_schedule(pabd_batch* b, const pabd_schedule* sch) {
  if (!b || !sch) return fail(PABD_E_INVALID, "null argument");
  if (sch->tile_bodies != 0 && sch->tile_bodies != 32 && sch->tile_bodies != 64 && sch->tile_bodies != 128 &&
      sch->tile_bodies != 256)
    return fail(PABD_E_INVALID, "tile size must be 0, 32, 64, 128 or 256");
  if (!valid_lanes(sch->contact_lanes)) return fail(PABD_E_INVALID, "contact lanes must be 1, 2, 4, 8 or 16");
  if (!valid_waves(sch->group_waves)) return fail(PABD_E_INVALID, "wavefronts per workgroup must be 1, 2 or 4");
  if (sch->tile_bodies != 0) {
    pabd_status st = pabd_batch_set_tile(b, sch->tile_bodies);
    if (st != PABD_OK) return st;
  }
  if (sch->contact_lanes != b->contact_lanes || sch->group_waves != b->group_waves) {
    API_HIP(hipStreamSynchronize(b->stream));
    b->contact_lanes = sch->contact_lanes;
    b->group_waves = sch->group_waves;
    b->dirty = true;  // new wave table; the changed launch recaptures the graph
  }
  return PABD_OK;
}

pabd_status pabd_batch_tune(pabd_batch* b, int32_t flags, pabd_schedule* out) {
  if (!b) return fail(PABD_E_INVALID, "null batch");
  // the workload's shape, whatever the current placement: scenes the tile
  // kernel can take, contact scenes and other scenes (both always on the flat
  // path), and the largest contact capacity
  long long tileable = 0, contact = 0, other = 0;
  int largest = 0, ccap = 0;
  for (const Slot& s : b->slots) {
    if (!s.used) continue;
    if (s.hs->contact) {
      contact += s.n;
      ccap = std::max(ccap, s.hs->ccap);
    } else if (!s.hs->driven && !s.hs->variable) {
      tileable += s.n;
      largest = std::max(largest, s.n);
    } else {
      other += s.n;
    }
  }
  int tile_class = 0;
  if (largest > 0) {
    tile_class = 512;
    for (int t : {32, 64, 128, 256})
      if (t >= largest) {
        tile_class = t;
        break;
      }
  }
  TuneKey key;
  key.arch = device_arch();
  key.precision = b->precision;
  key.kind = 0;
  key.bucket[0] = bit_length(tileable);
  key.bucket[1] = tile_class;
  key.bucket[2] = bit_length(contact);
  key.bucket[3] = bit_length(other);
  key.bucket[4] = bit_length(ccap);
  pabd_status st;
  if (!(flags & PABD_TUNE_FORCE)) {
    pabd_schedule hit;
    bool found = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = tune_cache().find(key);
      if (it != tune_cache().end()) {
        hit = it->second;
        found = true;
      }
    }
    if (found) {
      hit.from_cache = 0;
      if ((st = pabd_batch_set_schedule(b, &hit)) != PABD_OK) return st;
      if ((st = pabd_batch_get_schedule(b, out ? out : &hit)) != PABD_OK) return st;
      if (out) out->from_cache = 1;
      return PABD_OK;
    }
  }
  const long long substeps0 = b->substeps;
  std::vector<char> snap;
  int n = 0, ne = 0;  // extent of the saved state (the scenes as placed when it was saved)
  auto save = [&]() {
    batch_extent(b, &n, &ne);
    return b->eng->snapshot(n, ne, snap, b->stream, false);
  };
  // whole steps (one graph replay each), timed from the saved state
  auto timed = [&](double* ms) {
    return time_steps(b->stream, 4, [&]() { return pabd_batch_steps(b, 1, nullptr); }, ms);
  };
  auto restore = [&]() {
    b->substeps = substeps0;
    return b->eng->snapshot(n, ne, snap, b->stream, true);
  };
  // 1. tile size.  With only scenes the tile kernel takes, the sizes that hold
  // them all, on the tile kernel alone; with other scenes beside them, every
  // size on whole steps (a smaller tile moves the larger chains to the flat
  // path, whose time then counts too).  A repack keeps every record bit for
  // bit, so each candidate starts from the same state.
  if (tileable > 0 && contact + other == 0) {
    int t = 0;
    if ((st = pabd_batch_autotune(b, &t)) != PABD_OK) return st;
  } else if (tileable > 0) {
    double best_t = 1e300;
    const int start = b->tile_bodies;
    int best = start;
    int order[4] = {start, 0, 0, 0}, no = 1;
    for (int t : {32, 64, 128, 256})
      if (t != start) order[no++] = t;
    for (int t : order) {
      // only sizes whose placement surely fits: the flat-path bodies within the
      // flat pool, the tiled ones within half the tile pool
      long long flat_n = 0, tiled_n = 0;
      for (const Slot& sl : b->slots) {
        if (!sl.used) continue;
        const bool tl = !sl.hs->contact && !sl.hs->driven && !sl.hs->variable && sl.n > 0 && sl.n <= t;
        (tl ? tiled_n : flat_n) += std::max(1, sl.n);
      }
      if (flat_n > b->n_stream || 2 * tiled_n > (long long)b->caps.n - b->n_stream) continue;
      if (t != b->tile_bodies && (st = batch_repack(b, t)) != PABD_OK) return st;
      API_HIP(hipDeviceSynchronize());
      if ((st = save()) != PABD_OK) return st;
      double dt = 1e300;
      for (int round = 0; round < 3; ++round) {
        double ms = 0.0;
        if ((st = timed(&ms)) != PABD_OK) return st;
        if ((st = restore()) != PABD_OK) return st;
        dt = std::min(dt, ms);
      }
      if (t == start ? dt < best_t : dt < (1.0 - kTuneMargin) * best_t) {
        best_t = dt;
        best = t;
      }
    }
    if (best != b->tile_bodies && (st = batch_repack(b, best)) != PABD_OK) return st;
    b->tile_auto = false;
  }
  // 2. the flat path (its scenes depend on the tile size just chosen)
  if (b->dirty) {
    if ((st = batch_tables(b)) != PABD_OK) return st;
    b->dirty = false;
  }
  long long flat_contact = 0, flat_other = 0;
  for (const Slot& s : b->slots)
    if (s.used && !s.tiled && !s.resident) (s.contact ? flat_contact : flat_other) += s.n;
  if (flat_contact + flat_other > 0) {
    API_HIP(hipDeviceSynchronize());
    if ((st = save()) != PABD_OK) return st;
    int cl = b->contact_lanes, gw = b->group_waves;
    auto apply = [&](int c, int g) {
      pabd_schedule sc{0, c, g, 0};
      (void)pabd_batch_set_schedule(b, &sc);
    };
    if ((st = search_flat(flat_contact > 0, &cl, &gw, apply, timed, restore)) != PABD_OK) return st;
  }
  pabd_schedule best;
  if ((st = pabd_batch_get_schedule(b, &best)) != PABD_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache()[key] = best;
  }
  if (out) *out = best;
  return PABD_OK;
}

pabd_status pabd_scene_get_schedule(const pabd_scene* s, pabd_schedule* out) {
  if (!s || !out) return fail(PABD_E_INVALID, "null argument");
  out->tile_bodies = 0;
  s->eng->get_schedule(&out->contact_lanes, &out->group_waves);
  out->from_cache = 0;
  return PABD_OK;
}

pabd_status pabd_scene_set_schedule(pabd_scene* s, const pabd_schedule* sch) {
  if (!s || !sch) return fail(PABD_E_INVALID, "null argument");
  if (!valid_lanes(sch->contact_lanes)) return fail(PABD_E_INVALID, "contact lanes must be 1, 2, 4, 8 or 16");
  if (!valid_waves(sch->group_waves)) return fail(PABD_E_INVALID, "wavefronts per workgroup must be 1, 2 or 4");
  int cl = 0, gw = 0;
  s->eng->get_schedule(&cl, &gw);
  if (cl != sch->contact_lanes || gw != sch->group_waves) {
    API_HIP(hipStreamSynchronize(s->stream));
    s->eng->set_schedule(sch->contact_lanes, sch->group_waves);
    s->graph.reset();  // the captured step launches the old schedule
  }
  return PABD_OK;
}

pabd_status pabd_scene_tune(pabd_scene* s, int32_t flags, pabd_schedule* out) {
  if (!s) return fail(PABD_E_INVALID, "null scene");
  pabd_status st;
  // a scene whose whole step runs in the resident kernel has no flat-path
  // launch to tune
  if ((s->resident && !s->history) || s->hs.n == 0) {
    pabd_schedule cur;
    if ((st = pabd_scene_get_schedule(s, &cur)) != PABD_OK) return st;
    if (out) *out = cur;
    return PABD_OK;
  }
  TuneKey key;
  key.arch = device_arch();
  key.precision = s->precision;
  key.kind = 1;
  key.bucket[0] = bit_length(s->hs.n);
  key.bucket[1] = s->hs.contact ? 1 : 0;
  key.bucket[2] = bit_length(s->hs.contact ? s->hs.ccap : 0);
  if (!(flags & PABD_TUNE_FORCE)) {
    pabd_schedule hit;
    bool found = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = tune_cache().find(key);
      if (it != tune_cache().end()) {
        hit = it->second;
        found = true;
      }
    }
    if (found) {
      if ((st = pabd_scene_set_schedule(s, &hit)) != PABD_OK) return st;
      if (out) {
        if ((st = pabd_scene_get_schedule(s, out)) != PABD_OK) return st;
        out->from_cache = 1;
      }
      return PABD_OK;
    }
  }
  API_HIP(hipDeviceSynchronize());
  std::vector<char> snap;
  const int n = std::max(1, s->hs.n), ne = std::max(1, s->hs.ne);
  if ((st = s->eng->snapshot(n, ne, snap, s->stream, false)) != PABD_OK) return st;
  int cl = 0, gw = 0;
  s->eng->get_schedule(&cl, &gw);
  auto apply = [&](int c, int g) {
    pabd_schedule sc{0, c, g, 0};
    (void)pabd_scene_set_schedule(s, &sc);
  };
  auto timed = [&](double* ms) {
    return time_steps(s->stream, 4, [&]() { return pabd_scene_step(s, 1, nullptr); }, ms);
  };
  auto restore = [&]() { return s->eng->snapshot(n, ne, snap, s->stream, true); };
  if ((st = search_flat(s->hs.contact, &cl, &gw, apply, timed, restore)) != PABD_OK) return st;
  pabd_schedule best;
  if ((st = pabd_scene_get_schedule(s, &best)) != PABD_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache()[key] = best;
  }
  if (out) *out = best;
  return PABD_OK;
}

// streaming copy, 16 bytes per lane per step, grid-stride
__global__ void __launch_bounds__(256) k_copy_probe(const float4* __restrict__ src, float4* __restrict__ dst,
                                                    size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

pabd_status pabd_hbm_copy_probe(size_t bytes, int32_t reps, double* gbps, double* avg_ms) {
  if (reps < 1 || bytes < 16) return fail(PABD_E_INVALID, "bad probe arguments");
  if (pabd_device_count() < 1) return fail(PABD_E_DEVICE, "no HIP device");
  const size_t n = bytes / 16;
  // every resource is released on every path, failures included
  struct Res {
    float4 *a = nullptr, *b = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Res() {
      if (st) (void)hipStreamSynchronize(st);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      if (a) (void)hipFree(a);
      if (b) (void)hipFree(b);
      if (st) (void)hipStreamDestroy(st);
    }
  } r;
  API_HIP(hipStreamCreateWithFlags(&r.st, hipStreamNonBlocking));
  if (hipMalloc(&r.a, n * 16) != hipSuccess || hipMalloc(&r.b, n * 16) != hipSuccess)
    return fail(PABD_E_OOM, "probe allocation failed");
  API_HIP(hipMemsetAsync(r.a, 0, n * 16, r.st));
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
  const dim3 grid((unsigned)std::min<size_t>((n + 255) / 256, (size_t)cus * 16)), block(256);
  hipLaunchKernelGGL(k_copy_probe, grid, block, 0, r.st, (const float4*)r.a, r.b, n);
  API_HIP(hipEventCreate(&r.e0));
  API_HIP(hipEventCreate(&r.e1));
  API_HIP(hipEventRecord(r.e0, r.st));
  for (int k = 0; k < reps; ++k) hipLaunchKernelGGL(k_copy_probe, grid, block, 0, r.st, (const float4*)r.a, r.b, n);
  API_HIP(hipEventRecord(r.e1, r.st));
  API_HIP(hipEventSynchronize(r.e1));
  float ms = 0.f;
  API_HIP(hipEventElapsedTime(&ms, r.e0, r.e1));
  const double per = (double)ms / reps;
  if (avg_ms) *avg_ms = per;
  if (gbps) *gbps = 2.0 * (double)(n * 16) / (per * 1e-3) / 1e9;
  return PABD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free run (pabd_scene_run_noalloc)
// ---------------------------------------------------------------------------

// Device memory of pabd_scene_run_noalloc: one file-scope array that each GPU
// the library runs on holds until the process ends.  In host code this name is
// a host-side stand-in, not a device address: host code uses the address that
// hipGetSymbolAddress gives for the current device (scratch_on_device), never
// the name itself.
static __device__ __align__(256) unsigned char scratch[PABD_NOALLOC_SCRATCH_BYTES];

namespace {

// per device: the address of its copy of `scratch`, looked up once with that
// device current
struct ScratchTable {
  std::mutex m;
  std::vector<void*> addr;
};

ScratchTable& scratch_table() {
  static ScratchTable t;
  return t;
}

pabd_status scratch_on_device(void** out) {
  int dev = 0;
  API_HIP(hipGetDevice(&dev));
  ScratchTable& t = scratch_table();
  std::lock_guard<std::mutex> lock(t.m);
  if ((int)t.addr.size() <= dev) t.addr.resize((size_t)dev + 1, nullptr);
  if (!t.addr[dev]) {
    void* p = nullptr;
    API_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(PABD_E_DEVICE, "hipGetSymbolAddress gave no address for the scratch array");
    t.addr[dev] = p;
  }
  *out = t.addr[dev];
  return PABD_OK;
}

// bump allocation from the scratch array, 256-byte aligned; NULL once full
struct Bump {
  char* base;
  size_t cap, used, asked;
};

void* bump_alloc(size_t bytes, void* ctx) {
  Bump* b = static_cast<Bump*>(ctx);
  const size_t off = (b->used + 255) / 256 * 256;
  b->asked = off + bytes;
  if (b->asked > b->cap) return nullptr;
  b->used = b->asked;
  return b->base + off;
}

void bump_release(void*, void*) {}

}  // namespace

extern "C" {

pabd_status pabd_scene_run_noalloc(const pabd_scene_desc* desc, int32_t nsteps, double* c, double* A,
                                   double* v, double* w, void* hip_stream) {
  if (nsteps < 0) return fail(PABD_E_INVALID, "negative step count");
  HostScene hs;
  std::string why = build_host_scene(desc, hs);
  if (!why.empty()) return fail(PABD_E_INVALID, why);
  if (pabd_device_count() < 1) return fail(PABD_E_DEVICE, "no HIP device");
  void* base = nullptr;
  pabd_status st = scratch_on_device(&base);
  if (st != PABD_OK) return st;
  hipStream_t stream = (hipStream_t)hip_stream;
  // the previous call on this stream may still be reading the scratch
  API_HIP(hipStreamSynchronize(stream));
  Bump bump{static_cast<char*>(base), (size_t)PABD_NOALLOC_SCRATCH_BYTES, 0, 0};
  DeviceAllocator mem;
  mem.alloc = bump_alloc;
  mem.release = bump_release;
  mem.ctx = &bump;
  std::unique_ptr<EngineBase> eng = make_engine(desc->precision);
  eng->use_memory(mem);
  Caps cp;
  cp.n = std::max(1, hs.n);
  cp.e = std::max(1, hs.ne);
  cp.s = 1;
  cp.p = std::max(1, (int)hs.planes.size() / 4);
  cp.dr = std::max(1, (int)hs.drv_end_i.size());
  cp.contacts = hs.contact;
  cp.cslots = (long long)cp.n * hs.ccap;
  // every array is taken before anything is written, so a scene that does not
  // fit is turned away before the device is touched
  st = eng->allocate(cp);
  if (st == PABD_E_OOM)
    return fail(PABD_E_OOM, "the scene needs more than the " + std::to_string((size_t)PABD_NOALLOC_SCRATCH_BYTES) +
                                " bytes of the library's static scratch (at least " + std::to_string(bump.asked) +
                                " bytes)");
  if (st != PABD_OK) return fail(st, eng->error());
  hs.params.steps_total = INT_MAX;
  // the same path as the plain scene's (pabd_scene_step)
  const bool resident = hs.n > 0 && hs.n <= eng->resident_max(hs.contact);
  hs.params.resident = resident ? 1 : 0;
  st = eng->upload(hs, 0, 0, 0, 0, 0, stream);
  if (st != PABD_OK) return fail(st, eng->error());
  if (resident) {
    st = hs.contact ? eng->set_resident({0}, {}, hs.variable, stream)
                    : eng->set_resident({}, {0}, hs.variable, stream);
    if (st != PABD_OK) return fail(st, eng->error());
  }
  eng->factor(stream);
  const int grid[2] = {hs.contact ? 1 : 0, hs.contact ? 0 : 1};
  for (int k = 0; k < nsteps && hs.n > 0; ++k)
    eng->flat_step(0, std::max(1, hs.n), 1, hs.params.iters, hs.contact, (int)hs.drv_end_i.size(), false,
                   true, stream, nullptr, nullptr, 0, resident ? grid : nullptr, !resident);
  API_HIP(hipGetLastError());
  st = eng->read_bodies(0, hs.n, c, A, v, w, stream);
  if (st != PABD_OK) return st;
  int health = 0;
  API_HIP(hipMemcpy(&health, eng->health_ptr(), sizeof(int), hipMemcpyDeviceToHost));
  if (health & 1) return fail(PABD_E_DIVERGED, "non-finite state");
  if (health & 2) return fail(PABD_E_DIVERGED, "contact capacity exceeded");
  return PABD_OK;
}

}  // extern "C"
