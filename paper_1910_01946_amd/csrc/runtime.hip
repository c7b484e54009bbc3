// Host runtime of the library: RVE set-up, the Newton / conjugate-gradient increment
// loop of Section 2.2 (eqs. 15-18), commit, Nye tensor and GND densities, and the C ABI
// declared in include/rve.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <memory>
#include <mutex>
#include <thread>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/rve.h"
#include "adjoint.h"
#include "kernels.h"
#include "spectral.h"

namespace rve {

// ------------------------------------------------------------------------------------
// errors
// ------------------------------------------------------------------------------------
static thread_local std::string g_last_error;

struct Error : std::runtime_error {
  int32_t code;
  Error(int32_t c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHECK(x)                                                                                  \
  do {                                                                                               \
    hipError_t e_ = (x);                                                                             \
    if (e_ != hipSuccess)                                                                            \
      throw Error(e_ == hipErrorOutOfMemory ? RVE_ENOMEM : RVE_EDEVICE,                              \
                  std::string(#x) + ": " + hipGetErrorString(e_));                                   \
  } while (0)

static void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(RVE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Settings read from the environment once per process (std::call_once), before any
// worker thread exists, so that no thread races on their first read:
//   RVE_TRACE=1      one line per Newton iteration on stderr;
//   RVE_PREDICT=0    start every local solve from the previous slip increments instead of
//                    their first-order prediction (same converged result);
//   RVE_PLANE=0      the three-pass (x, y, z) spectral kernels even where the plane kernels
//                    fit (both are kept and tested);
//   RVE_TANGENT16=0  the mixed form's tangent copy in FP32 instead of scaled FP16;
//   RVE_TZ=t         cap on the z-pass tile width;
//   RVE_WORKERS=w    host threads driving RVEs concurrently (default 8).
struct Settings {
  bool trace = false, predict = true, plane = true, tangent16 = true;
  int tz_cap = 0, workers = 8;
};
static const Settings& settings() {
  static Settings s;
  static std::once_flag once;
  std::call_once(once, []() {
    auto env = [](const char* name) -> const char* {
      const char* e = std::getenv(name);
      return (e && e[0]) ? e : nullptr;
    };
    if (const char* e = env("RVE_TRACE")) s.trace = e[0] != '0';
    if (const char* e = env("RVE_PREDICT")) s.predict = e[0] != '0';
    if (const char* e = env("RVE_PLANE")) s.plane = e[0] != '0';
    if (const char* e = env("RVE_TANGENT16")) s.tangent16 = e[0] != '0';
    if (const char* e = env("RVE_TZ")) s.tz_cap = std::max(1, std::atoi(e));
    if (const char* e = env("RVE_WORKERS")) s.workers = std::max(1, std::atoi(e));
  });
  return s;
}
static bool trace_on() { return settings().trace; }
static bool prediction_enabled() { return settings().predict; }
static bool plane_enabled() { return settings().plane; }
static bool tangent16_enabled() { return settings().tangent16; }

// ------------------------------------------------------------------------------------
// host-side tables (independent of any other implementation)
// ------------------------------------------------------------------------------------
static const int kPlane[4][3] = {{1, 1, 1}, {-1, 1, 1}, {1, -1, 1}, {1, 1, -1}};
static const int kDir[12][3] = {{0, 1, -1}, {-1, 0, 1}, {1, -1, 0}, {0, 1, -1}, {1, 0, 1}, {1, 1, 0},
                                {0, 1, 1},  {1, 0, -1}, {1, 1, 0},  {0, 1, 1},  {1, 0, 1}, {1, -1, 0}};

static int dot3i(const int* a, const int* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// q^{ab} from the six Table 1 coefficients (self, coplanar, collinear, Hirth, glissile, Lomer)
static void interaction_matrix(const double* coef, double* q) {
  for (int a = 0; a < 12; ++a)
    for (int b = 0; b < 12; ++b) {
      const int* na = kPlane[a / 3];
      const int* nb = kPlane[b / 3];
      const int* sa = kDir[a];
      const int* sb = kDir[b];
      int cls;
      if (a == b) cls = 0;
      else if (a / 3 == b / 3) cls = 1;
      else {
        const int cx = sa[1] * sb[2] - sa[2] * sb[1], cy = sa[2] * sb[0] - sa[0] * sb[2],
                  cz = sa[0] * sb[1] - sa[1] * sb[0];
        if (cx == 0 && cy == 0 && cz == 0) cls = 2;
        else if (dot3i(sa, sb) == 0) cls = 3;
        else {
          int j[3];
          for (int i = 0; i < 3; ++i) j[i] = sa[i] + sb[i];
          if (dot3i(j, j) != 2)
            for (int i = 0; i < 3; ++i) j[i] = sa[i] - sb[i];
          cls = (dot3i(j, na) == 0 || dot3i(j, nb) == 0) ? 4 : 5;
        }
      }
      q[12 * a + b] = coef[cls];
    }
}

// A (9 x 18): edge columns vec(b (x) t), t = m x b; screw columns vec(b (x) b); A^+ = A^T (A A^T)^{-1}
static void segment_pinv(double* Aplus, int* screw_of) {
  double A[9][18];
  double sdir[6][3];
  int nscrew = 0;
  for (int a = 0; a < 12; ++a) {
    double b[3], m[3], t[3];
    const double ib = 1.0 / std::sqrt(2.0), im = 1.0 / std::sqrt(3.0);
    for (int i = 0; i < 3; ++i) {
      b[i] = kDir[a][i] * ib;
      m[i] = kPlane[a / 3][i] * im;
    }
    t[0] = m[1] * b[2] - m[2] * b[1];
    t[1] = m[2] * b[0] - m[0] * b[2];
    t[2] = m[0] * b[1] - m[1] * b[0];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) A[3 * i + j][a] = b[i] * t[j];
    int found = -1;
    for (int s = 0; s < nscrew; ++s) {
      const double d = std::fabs(sdir[s][0] * b[0] + sdir[s][1] * b[1] + sdir[s][2] * b[2]);
      if (std::fabs(d - 1.0) < 1e-12) found = s;
    }
    if (found < 0) {
      for (int i = 0; i < 3; ++i) sdir[nscrew][i] = b[i];
      found = nscrew++;
    }
    screw_of[a] = found;
  }
  for (int s = 0; s < 6; ++s)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) A[3 * i + j][12 + s] = sdir[s][i] * sdir[s][j];
  // M = A A^T, invert by Gauss-Jordan with partial pivoting
  double M[9][18];
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      double s = 0.0;
      for (int k = 0; k < 18; ++k) s += A[i][k] * A[j][k];
      M[i][j] = s;
      M[i][9 + j] = (i == j) ? 1.0 : 0.0;
    }
  for (int c = 0; c < 9; ++c) {
    int piv = c;
    for (int r = c + 1; r < 9; ++r)
      if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
    for (int k = 0; k < 18; ++k) std::swap(M[c][k], M[piv][k]);
    const double ip = 1.0 / M[c][c];
    for (int k = 0; k < 18; ++k) M[c][k] *= ip;
    for (int r = 0; r < 9; ++r)
      if (r != c) {
        const double f = M[r][c];
        for (int k = 0; k < 18; ++k) M[r][k] -= f * M[c][k];
      }
  }
  // A^+ (18 x 9) = A^T M^{-1}
  for (int s = 0; s < 18; ++s)
    for (int c = 0; c < 9; ++c) {
      double v = 0.0;
      for (int k = 0; k < 9; ++k) v += A[k][s] * M[k][9 + c];
      Aplus[s * 9 + c] = v;
    }
}

static void quat_to_R(const double* q_in, double* R) {
  double w = q_in[0], x = q_in[1], y = q_in[2], z = q_in[3];
  const double n = std::sqrt(w * w + x * x + y * y + z * z);
  w /= n; x /= n; y /= n; z /= n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static MatDev make_material(const rve_material& m) {
  auto finite_pos = [](double v) { return std::isfinite(v) && v > 0.0; };
  if (!finite_pos(m.C11) || !finite_pos(m.C44) || !std::isfinite(m.C12) || m.C11 - m.C12 <= 0.0 ||
      m.C11 + 2 * m.C12 <= 0.0)
    throw Error(RVE_EINVAL, "elastic constants are not positive definite");
  if (!finite_pos(m.burgers) || !finite_pos(m.gamma0_dot) || !finite_pos(m.m_rate) || !finite_pos(m.K_sim) ||
      !(std::isfinite(m.y_c) && m.y_c >= 0.0) || !(std::isfinite(m.c_gnd) && m.c_gnd >= 0.0))
    throw Error(RVE_EINVAL, "dislocation or flow-rule parameter not positive");
  MatDev d;
  std::memset(&d, 0, sizeof(d));
  d.C11 = m.C11;
  d.C12 = m.C12;
  d.C44 = m.C44;
  d.mu = m.mu > 0 ? m.mu : 3.0 * m.C44 * (m.C11 - m.C12) / (m.C11 - m.C12 + 4.0 * m.C44);
  d.burgers = m.burgers;
  d.y_c = m.y_c;
  d.K_sim = m.K_sim;
  d.gamma0_dot = m.gamma0_dot;
  d.n_exp = 1.0 / m.m_rate;
  d.c_gnd = m.c_gnd;
  d.hardening = m.hardening ? 1 : 0;
  interaction_matrix(m.q, d.q);
  double rowsum = 0.0;
  for (int b = 0; b < 12; ++b) rowsum += d.q[b];
  double rho0 = m.rho0;
  if (!(rho0 > 0.0)) {
    if (!finite_pos(m.tau0)) throw Error(RVE_EINVAL, "need tau0 > 0 or rho0 > 0");
    rho0 = std::pow(m.tau0 / (d.mu * d.burgers), 2) / rowsum;
  }
  if (!std::isfinite(rho0) || rho0 <= 0.0) throw Error(RVE_EINVAL, "initial density must be positive");
  d.tau_c_frozen = d.mu * d.burgers * std::sqrt(rowsum * rho0);
  d.pad = 0;
  segment_pinv(d.Aplus, d.screw_of);
  // keep rho0 for the state initialisation in an unused slot
  return d;
}

static double initial_rho0(const rve_material& m, const MatDev& d) {
  if (m.rho0 > 0.0) return m.rho0;
  double rowsum = 0.0;
  for (int b = 0; b < 12; ++b) rowsum += d.q[b];
  return std::pow(m.tau0 / (d.mu * d.burgers), 2) / rowsum;
}

// ------------------------------------------------------------------------------------
// grid plans
// ------------------------------------------------------------------------------------
static AxisPlan make_axis(int n) {
  AxisPlan a;
  a.n = n;
  a.nrad = 0;
  int m = n;
  const int order[5] = {8, 4, 2, 3, 5};
  for (int r : order)
    while (m % r == 0 && m > 1) {
      if (a.nrad >= 8) throw Error(RVE_EINVAL, "grid size has too many factors");
      a.rad[a.nrad++] = r;
      m /= r;
    }
  if (m != 1) throw Error(RVE_EINVAL, "grid sizes must have prime factors 2, 3 and 5 only");
  a.code = 0;
  for (int s = 0; s < a.nrad; ++s) a.code |= (uint32_t)a.rad[s] << (4 * s);
  return a;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  void alloc(size_t b) {
    if (p) {
      (void)hipFree(p);
      p = nullptr;
    }
    bytes = b;
    if (b) HIPCHECK(hipMalloc(&p, b));
  }
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

struct Plan {
  GridPlan g;
  DevBuf tw[3], E[3];
};

// Sizes, radix plans, tile widths and divisors of a grid (no tables, nothing allocated).
static void plan_geometry(GridPlan& g, const int n[3], int tz_choice = 0, int tz3_choice = 0) {
  for (int d = 0; d < 3; ++d)
    if (n[d] < 1 || n[d] > 256) throw Error(RVE_EINVAL, "grid sizes must lie in 1..256");
  g.nx = n[0];
  g.ny = n[1];
  g.nz = n[2];
  g.nxh = n[0] / 2 + 1;
  g.nvox = (int64_t)n[0] * n[1] * n[2];
  g.nspec = (int64_t)g.nxh * n[1] * n[2];
  g.ax = make_axis(n[0]);
  g.ay = make_axis(n[1]);
  g.az = make_axis(n[2]);
  // rows per x block: even, ly * nx <= max(256, 2 nx)
  int ly = std::max(2, (std::max(256, 2 * g.nx) / g.nx) & ~1);
  const int ny_even = (g.ny + 1) & ~1;
  g.ly = std::min(ly, ny_even);
  g.ty = std::min(16, g.nxh);
  if (g.ny * g.ty > 16 * 256) g.ty = (16 * 256) / g.ny;
  // kx columns per z-pass block: nz * tz <= 256, i.e. at most 9 points per thread of a
  // 256-thread block (the z-pass transform is compiled for that bound)
  g.tz = std::max(1, std::min(g.nxh, 256 / g.nz));
  // the three-component z pass: the same columns per block by default (a third of the
  // work per block), up to three times as many (the same points per thread)
  g.tz3 = g.tz;
  if (tz_choice > 0) g.tz = std::min(g.tz, tz_choice);
  if (tz3_choice > 0) g.tz3 = std::max(1, std::min(std::min(g.nxh, 768 / g.nz), tz3_choice));
  if (settings().tz_cap > 0) {
    g.tz = std::min(g.tz, settings().tz_cap);
    g.tz3 = std::min(g.tz3, settings().tz_cap);
  }
  g.fnx = make_fastdiv(g.nx);
  g.fnxh = make_fastdiv(g.nxh);
  g.fnz = make_fastdiv(g.nz);
  g.ftz = make_fastdiv(g.tz);
  g.ftz3 = make_fastdiv(g.tz3);
  g.freq = FREQ_ROTATED;
}

// Tile widths chosen by the autotuner, per (grid, spectral precision), for the whole process.
struct TuneKey {
  int n0, n1, n2, fp32;
  bool operator==(const TuneKey& o) const { return n0 == o.n0 && n1 == o.n1 && n2 == o.n2 && fp32 == o.fp32; }
};
struct TunedTiles {
  int tz = 0, tz3 = 0;  // 0: not tuned
};
static std::mutex g_tune_mu;
static std::vector<std::pair<TuneKey, TunedTiles>> g_tuned_tz;

static TunedTiles tuned_tz(const int n[3], bool fp32) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const TuneKey k{n[0], n[1], n[2], fp32 ? 1 : 0};
  for (const auto& e : g_tuned_tz)
    if (e.first == k) return e.second;
  return TunedTiles{};
}

// st: the stream that uploads the tables (stream-ordered, then synchronised).  Plans built
// while other threads may be capturing CG graphs (a worker's first FP64 use) must pass their
// RVE's stream: a synchronous copy runs on the legacy stream, which a capture in progress on
// another stream forbids.
static void build_plan(Plan& P, const int n[3], bool fp32, bool autotune = false, int freq = FREQ_ROTATED,
                       hipStream_t st = nullptr) {
  GridPlan& g = P.g;
  const TunedTiles tt = autotune ? tuned_tz(n, fp32) : TunedTiles{};
  plan_geometry(g, n, tt.tz, tt.tz3);
  g.freq = freq;
  // table of roots: tw[k] = exp(-2 pi i k / n); E[q] = exp(+2 pi i q / n) exact at quarter turns
  for (int d = 0; d < 3; ++d) {
    const int m = n[d];
    std::vector<double> tw(2 * m), E(2 * m);
    for (int k = 0; k < m; ++k) {
      const long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)m;
      double c = (double)cosl(ang), s = (double)sinl(ang);
      if (k == 0) { c = 1; s = 0; }
      if (2 * k == m) { c = -1; s = 0; }
      if (4 * k == m) { c = 0; s = 1; }
      if (4 * k == 3 * m) { c = 0; s = -1; }
      tw[2 * k] = c;
      tw[2 * k + 1] = -s;
      E[2 * k] = c;
      E[2 * k + 1] = s;
    }
    auto put = [&](void* dst, const void* src, size_t bytes) {
      if (st) {
        HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
        HIPCHECK(hipStreamSynchronize(st));  // the host vectors end with this iteration
      } else {
        HIPCHECK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
      }
    };
    if (fp32) {
      std::vector<float> twf(2 * m);
      for (int i = 0; i < 2 * m; ++i) twf[i] = (float)tw[i];
      P.tw[d].alloc(sizeof(float) * 2 * m);
      put(P.tw[d].p, twf.data(), sizeof(float) * 2 * m);
    } else {
      P.tw[d].alloc(sizeof(double) * 2 * m);
      put(P.tw[d].p, tw.data(), sizeof(double) * 2 * m);
    }
    P.E[d].alloc(sizeof(double) * 2 * m);
    put(P.E[d].p, E.data(), sizeof(double) * 2 * m);
  }
  g.twx = P.tw[0].p;
  g.twy = P.tw[1].p;
  g.twz = P.tw[2].p;
  g.Ex = P.E[0].p;
  g.Ey = P.E[1].p;
  g.Ez = P.E[2].p;
}

static size_t tsize(bool fp32) { return fp32 ? 4 : 8; }


// ------------------------------------------------------------------------------------
// one RVE on the device
// ------------------------------------------------------------------------------------
// Precision-specific work buffers of one RVE (FP64 or FP32 spectral path).
struct Work {
  bool fp32 = false;
  bool ready = false;
  Plan plan;
  DevBuf K, xa, xb, xbest, r, p, q, y, spec;
  DevBuf w3;           // factorised projection: the three components w_i (T)
  bool plane = false;  // x/y transforms of one component plane in LDS (when it fits)
  bool g3 = false;     // CG iterations take the factorised projection
  bool k16 = false;    // FP32 work set with the plane path: tangent copy as scaled FP16 pairs
  bool k_ready = false;  // K holds the tangent of the last constitutive evaluation with tangent
  // captured CG chunks (one HIP graph each), by [tangent transposed][CG unknown xa or xb]
  hipGraphExec_t cg_graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  Work() = default;
  Work(const Work&) = delete;
  Work& operator=(const Work&) = delete;
  ~Work() {
    for (auto& row : cg_graph)
      for (hipGraphExec_t& e : row)
        if (e) (void)hipGraphExecDestroy(e);
  }
};

// Times the launches of the families in mask with HIP events that the kernel dispatch
// itself records at the kernel's start and end (on the launching stream), and accumulates
// launch count, duration and algorithmic bytes per family.
// Launches inside a conjugate-gradient solve carry the iteration they belong to (tag), so
// that the launches issued past the end of the solve (they return at once) are dropped.
struct EventTimer final : LaunchTimer {
  uint32_t mask = 0;
  int tag = -1;  // CG iteration of the launches being issued; -1 outside CG
  struct Rec {
    int family, tag;
    hipEvent_t a, b;
    int64_t bytes;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t open[KF_COUNT] = {}, close_[KF_COUNT] = {};
  int64_t launches[KF_COUNT] = {};
  double ms[KF_COUNT] = {}, bytes[KF_COUNT] = {};

  bool on(int f) const { return (mask >> f) & 1u; }
  hipEvent_t take() {
    if (pool.empty()) {
      // device-scope release: no system-scope cache writeback at the kernel's end, which
      // would otherwise lengthen the timed kernel itself
      hipEvent_t e;
      HIPCHECK(hipEventCreateWithFlags(&e, hipEventReleaseToDevice));
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  // The launch between begin() and end() records the two events at its own start and end.
  void begin(int f, hipStream_t) override {
    if (!on(f)) return;
    LaunchEvents& ev = pending_launch_events();
    ev.start = take();
    ev.stop = take();
    open[f] = ev.start;
    close_[f] = ev.stop;
  }
  void end(int f, int64_t b, hipStream_t) override {
    if (!on(f)) return;
    pending_launch_events() = LaunchEvents{};
    pending.push_back({f, tag, open[f], close_[f], b});
  }
  // Accumulate the recorded launches (their stream has been synchronised).  live_iters:
  // iterations the CG solve completed; its transform launches of later iterations, and its
  // vector-update launches after the one that found convergence, did no work.
  void resolve(int live_iters = 1 << 30) {
    for (const Rec& r : pending) {
      const bool live = r.tag < 0 || (r.family == KF_CG_PREP ? r.tag <= live_iters : r.tag < live_iters);
      if (live) {
        float t = 0.f;
        HIPCHECK(hipEventElapsedTime(&t, r.a, r.b));
        launches[r.family] += 1;
        ms[r.family] += t;
        bytes[r.family] += (double)r.bytes;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  void reset(uint32_t m) {
    mask = m;
    for (int f = 0; f < KF_COUNT; ++f) launches[f] = 0, ms[f] = 0.0, bytes[f] = 0.0;
  }
  ~EventTimer() override {
    for (const Rec& r : pending) (void)hipEventDestroy(r.a), (void)hipEventDestroy(r.b);
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// Algorithmic bytes of one launch (compulsory HBM traffic: every input read once, every
// output written once).  T = spectral precision, nv voxels, ns = nxh ny nz spectral points.
static int64_t bytes_mid(const GridPlan& g, bool fp32) { return 2 * 9 * 2 * (fp32 ? 4 : 8) * g.nspec; }
static int64_t bytes_cg_prep(const GridPlan& g, bool fp32, bool k16, bool first) {
  // r, q, K read and r, y written (first iteration: r, K read and y written); K: 81 entries,
  // or 41 pairs of FP16; grain id
  const int t = fp32 ? 4 : 8;
  return ((first ? 18 : 36) * t + (k16 ? 81 * 2 : 81 * t) + 4) * g.nvox;
}
static int64_t bytes_plane_fwd_cg(const GridPlan& g, bool fp32) {
  const int t = fp32 ? 4 : 8;
  return 9 * t * g.nvox + 9 * 2 * t * g.nspec;  // y read, spectrum written
}
static int64_t bytes_plane_inv_cg(const GridPlan& g, bool fp32, bool first) {
  // spectrum, r read; p, q, x read and written (first iteration: p, q written)
  const int t = fp32 ? 4 : 8;
  return 9 * 2 * t * g.nspec + (first ? 27 : 63) * t * g.nvox;
}
// factorised projection: y read and three spectra written; three spectra read and written;
// three spectra read and w written; w, r read, p, q, x read and written (first iteration: w,
// r read, p, q written)
static int64_t bytes_plane_div(const GridPlan& g, bool fp32) {
  const int t = fp32 ? 4 : 8;
  return 9 * t * g.nvox + 3 * 2 * t * g.nspec;
}
static int64_t bytes_mid3(const GridPlan& g, bool fp32) { return 2 * 3 * 2 * (fp32 ? 4 : 8) * g.nspec; }
static int64_t bytes_plane_inv3(const GridPlan& g, bool fp32) {
  const int t = fp32 ? 4 : 8;
  return 3 * 2 * t * g.nspec + 3 * t * g.nvox;
}
static int64_t bytes_cg_grad(const GridPlan& g, bool fp32, bool first) {
  const int t = fp32 ? 4 : 8;
  return (first ? 30 : 66) * t * g.nvox;
}
static int64_t bytes_plane_fwd_f64(const GridPlan& g, bool fp32) {
  return 9 * 8 * g.nvox + 9 * 2 * (fp32 ? 4 : 8) * g.nspec;  // FP64 field read, spectrum written
}
static int64_t bytes_plane_inv_resid(const GridPlan& g, bool fp32) {
  const int t = fp32 ? 4 : 8;
  return 9 * 2 * t * g.nspec + 27 * t * g.nvox;  // spectrum read; x, r, p written
}

struct RVE {
  Work w[2];     // [0] FP64, [1] FP32 (allocated on first use)
  int n[3];
  int64_t nvox = 0;
  double h = 0;
  double c11_rms = 0;  // rms over the voxels of C11 (sets the FP64 form's residual floor)
  int n_grains = 0;
  MatDev mat;
  double rho0 = 0;
  DevBuf d_mat, d_gid, d_R;
  // committed state
  DevBuf F, F_prev, Fp, rho_ssd, rho_gnd, nye, dg, P;
  // start-of-increment state of the last committed increment (for its reverse pass)
  DevBuf Fp_prev, rho_ssd_prev, rho_gnd_prev;
  double dt_last = 0.0;
  // work buffers of the reverse pass (allocated on first use)
  DevBuf adj_a9, adj_b9, adj_rgb, adj_theta;
  // work
  DevBuf F_work, F_try, P_work, dg_saved, cg, partial, blk;
  DevBuf dgdF;  // FP32 slip sensitivity d(dg)/dF_c, 108 x nvox, written with the tangent
  int64_t fp64_fallbacks = 0;
  hipStream_t stream = nullptr;   // each RVE runs on its own stream
  CGState* host_cg = nullptr;     // pinned copy of the CG scalars
  CGState* host_poll = nullptr;   // two pinned snapshots of the CG scalars, read by the chunk loop
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  EventTimer timer;               // optional launch timing
  Plan proj_plan;                 // FP64 projection of the Newton correction (mixed form)
  DevBuf proj_spec, x64;
  bool proj_ready = false;
  bool autotune = false;          // plans take the autotuned z-pass tile width
  int freq = FREQ_ROTATED;        // frequency scheme of the projection and the curl
  bool factorised = true;         // factorised projection in the CG iterations where it applies
  DevBuf d_C;                     // per-grain C11, C12, C44 (empty: the material's)
  LaunchTimer* tm() { return timer.mask ? &timer : nullptr; }
  ~RVE() {
    if (host_cg) (void)hipHostFree(host_cg);
    if (host_poll) (void)hipHostFree(host_poll);
    for (hipEvent_t e : poll_ev)
      if (e) (void)hipEventDestroy(e);
    if (stream) (void)hipStreamDestroy(stream);
  }
  bool have_prev = false;
  double Favg[9], Favg_prev[9], Pavg[9];
  double Fbar_prev[9];
  double Pbar_prev[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // stress targets of the last increment
  int64_t increments = 0;
};

struct Ctx {
  int device = 0;
  bool fp32 = false;
  int workers = 8;               // host threads driving RVEs concurrently
  bool use_graph = false;        // CG chunks as captured HIP graphs
  int freq = FREQ_ROTATED;       // frequency scheme of the projection and the curl
  bool factorised = true;        // factorised projection in the CG iterations where it applies
  int max_cutbacks = 0;          // halvings of the time step of a failed increment
  int max_continuation = 16;     // load-continuation stages of a failed FP64 attempt
  bool autotune = false;         // autotuned z-pass tile widths
  rve_options opt;
  hipStream_t stream = nullptr;  // caller's stream (optional)
  bool own_stream = false;
  std::vector<std::unique_ptr<RVE>> rves;
};

static void upload(DevBuf& b, const void* src, size_t bytes) {
  b.alloc(bytes);
  HIPCHECK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
}

static Work& work(RVE& R, bool fp32) {
  Work& w = R.w[fp32 ? 1 : 0];
  if (!w.ready) {
    w.fp32 = fp32;
    build_plan(w.plan, R.n, fp32, R.autotune, R.freq, R.stream);
    const int64_t nv = R.nvox;
    const size_t ts = tsize(fp32);
    // grouped layout: G groups of W entries per voxel (see tangent_index)
    // (an FP32 work set also holds the FP16 copy, TangentGroups<__half>::kStored <= 81 floats)
    w.K.alloc(ts * (fp32 ? TangentGroups<float>::kStored : TangentGroups<double>::kStored) * nv);
    w.xa.alloc(ts * 9 * nv);
    w.xb.alloc(ts * 9 * nv);
    w.xbest.alloc(ts * 9 * nv);
    w.r.alloc(ts * 9 * nv);
    w.p.alloc(ts * 9 * nv);
    w.q.alloc(ts * 9 * nv);
    w.spec.alloc(ts * 2 * 9 * w.plan.g.nspec);
    w.y.alloc(ts * 9 * nv);
    w.ready = true;
  }
  w.plane = plane_enabled() && plane_fits(w.plan.g, fp32);
  w.g3 = R.factorised && w.plane && factorised_fits(w.plan.g);
  if (w.g3 && !w.w3.p) w.w3.alloc(tsize(fp32) * 3 * (size_t)R.nvox);
  // (K is allocated at the FP32 size, which holds the FP16 pairs too)
  w.k16 = fp32 && w.plane && tangent16_enabled();
  return w;
}

static void prepare_correction(RVE& R);

static void init_rve(Ctx& C, RVE& R, const rve_desc& d) {
  for (int i = 0; i < 3; ++i) R.n[i] = d.n[i];
  R.autotune = C.autotune;
  R.nvox = (int64_t)d.n[0] * d.n[1] * d.n[2];
  if (!(std::isfinite(d.voxel_size) && d.voxel_size > 0)) throw Error(RVE_EINVAL, "voxel_size must be > 0");
  R.h = d.voxel_size;
  if (d.n_grains < 1 || !d.grain_of_voxel || !d.grain_quat) throw Error(RVE_EINVAL, "missing grain data");
  R.n_grains = d.n_grains;
  for (int64_t v = 0; v < R.nvox; ++v)
    if (d.grain_of_voxel[v] < 0 || d.grain_of_voxel[v] >= d.n_grains)
      throw Error(RVE_EINVAL, "grain id out of range at voxel " + std::to_string(v));
  std::vector<double> Rg(9 * (size_t)d.n_grains);
  for (int gi = 0; gi < d.n_grains; ++gi) {
    const double* q = d.grain_quat + 4 * gi;
    const double nn = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    if (!(std::isfinite(nn) && nn > 0)) throw Error(RVE_EINVAL, "bad quaternion");
    quat_to_R(q, &Rg[9 * gi]);
  }
  R.mat = make_material(d.material);
  R.rho0 = initial_rho0(d.material, R.mat);
  R.freq = C.freq;
  R.factorised = C.factorised;
  if (d.grain_elastic) {
    for (int gi = 0; gi < d.n_grains; ++gi) {
      const double* c = d.grain_elastic + 3 * gi;
      if (!(std::isfinite(c[0]) && std::isfinite(c[1]) && std::isfinite(c[2]) && c[2] > 0.0 && c[0] - c[1] > 0.0 &&
            c[0] + 2.0 * c[1] > 0.0))
        throw Error(RVE_EINVAL, "elastic constants of grain " + std::to_string(gi) + " are not positive definite");
    }
    upload(R.d_C, d.grain_elastic, sizeof(double) * 3 * (size_t)d.n_grains);
    double s2 = 0.0;
    for (int64_t v = 0; v < R.nvox; ++v) {
      const double c11 = d.grain_elastic[3 * d.grain_of_voxel[v]];
      s2 += c11 * c11;
    }
    R.c11_rms = std::sqrt(s2 / (double)R.nvox);
  } else {
    R.c11_rms = R.mat.C11;
  }
  upload(R.d_mat, &R.mat, sizeof(MatDev));
  upload(R.d_gid, d.grain_of_voxel, sizeof(int32_t) * R.nvox);
  upload(R.d_R, Rg.data(), sizeof(double) * Rg.size());
  const int64_t nv = R.nvox;
  const size_t f9 = sizeof(double) * 9 * nv, f12 = sizeof(double) * 12 * nv;
  std::vector<double> eye(9 * nv, 0.0), rho(12 * nv, R.rho0);
  for (int c = 0; c < 9; c += 4)
    for (int64_t v = 0; v < nv; ++v) eye[c * nv + v] = 1.0;
  upload(R.F, eye.data(), f9);
  upload(R.F_prev, eye.data(), f9);
  upload(R.Fp, eye.data(), f9);
  upload(R.rho_ssd, rho.data(), f12);
  R.rho_gnd.alloc(f12);
  HIPCHECK(hipMemset(R.rho_gnd.p, 0, f12));
  R.nye.alloc(f9);
  HIPCHECK(hipMemset(R.nye.p, 0, f9));
  R.dg.alloc(f12);
  HIPCHECK(hipMemset(R.dg.p, 0, f12));
  R.P.alloc(f9);
  HIPCHECK(hipMemset(R.P.p, 0, f9));
  upload(R.Fp_prev, eye.data(), f9);
  upload(R.rho_ssd_prev, rho.data(), f12);
  R.rho_gnd_prev.alloc(f12);
  HIPCHECK(hipMemset(R.rho_gnd_prev.p, 0, f12));
  R.F_work.alloc(f9);
  R.F_try.alloc(f9);
  R.P_work.alloc(f9);
  R.dg_saved.alloc(f12);
  R.dgdF.alloc(sizeof(float) * 108 * (size_t)nv);
  HIPCHECK(hipStreamCreateWithFlags(&R.stream, hipStreamNonBlocking));
  HIPCHECK(hipHostMalloc((void**)&R.host_cg, sizeof(CGState), hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void**)&R.host_poll, 2 * sizeof(CGState), hipHostMallocDefault));
  for (hipEvent_t& e : R.poll_ev) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  Work& w = work(R, C.fp32);
  if (C.fp32) prepare_correction(R);
  R.cg.alloc(sizeof(CGState));
  HIPCHECK(hipMemset(R.cg.p, 0, sizeof(CGState)));
  const int nb = std::max(std::max(xfwd_blocks(w.plan.g), 1024), std::max(9 * R.n[2], 2048));
  R.partial.alloc(sizeof(double) * 12 * nb);  // >= 3 x blocks of the x passes, 12 x colsum blocks
  R.blk.alloc(sizeof(int32_t) * (4 + nv));     // local-solve counters and work list
  for (int i = 0; i < 9; ++i) {
    R.Favg[i] = R.Favg_prev[i] = R.Fbar_prev[i] = (i % 4 == 0) ? 1.0 : 0.0;
    R.Pavg[i] = 0.0;
  }
}

// ------------------------------------------------------------------------------------
// building blocks of an increment
// ------------------------------------------------------------------------------------
struct LocalStats {
  int max_iters = 0;
  int failures = 0;
  int slow = 0;  // voxels handed to the continuation kernel
};

// predict: start the local solve from dg + (lam - lam_base) d(dg)/dF : dF, where dg and
// d(dg)/dF hold the converged solution of the previous call at F + lam_base dF.
static LocalStats run_constitutive(Ctx& C, RVE& R, Work& w, const double* F, const double* dF, double lam,
                                   double* F_out, double dt, bool tangent, bool predict = false,
                                   double lam_base = 0.0) {
  ConstArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nvox = R.nvox;
  a.gid = R.d_gid.as<int32_t>();
  a.grainR = R.d_R.as<double>();
  a.grainC = R.d_C.as<double>();
  a.mat = R.d_mat.as<MatDev>();
  a.F = F;
  a.dF = dF;
  a.lam = lam;
  a.F_out = F_out;
  a.Fp_n = R.Fp.as<double>();
  a.rho_ssd = R.rho_ssd.as<double>();
  a.rho_gnd = R.rho_gnd.as<double>();
  a.dg = R.dg.as<double>();
  a.P = R.P_work.as<double>();
  a.K = tangent ? w.K.p : nullptr;
  a.k_grouped = 1;
  a.k_inv_scale = w.k16 ? 1.0 / R.mat.C11 : 1.0;
  a.dt = dt;
  a.stats = R.blk.as<int32_t>();
  a.work = R.blk.as<int32_t>() + 4;
  a.dgdF = tangent ? R.dgdF.as<float>() : nullptr;
  a.predict = (predict && dF && prediction_enabled()) ? 1 : 0;
  a.lam_base = lam_base;
  launch_constitutive(a, !w.fp32 ? KT_F64 : (w.k16 ? KT_F16 : KT_F32), R.stream, R.tm());
  if (tangent) w.k_ready = true;
  check_launch("constitutive");
  int32_t st4[4];
  HIPCHECK(hipMemcpyAsync(st4, R.blk.p, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, R.stream));
  HIPCHECK(hipStreamSynchronize(R.stream));
  R.timer.resolve();
  LocalStats ls;
  ls.max_iters = st4[0];
  ls.failures = st4[1];
  ls.slow = st4[2];
  if (trace_on()) std::fprintf(stderr, "[rve] local solve: %d of %lld voxels on the continuation path, max it %d\n",
                               ls.slow, (long long)R.nvox, ls.max_iters);
  return ls;
}

// out = G(A) for a real FP64 field A (9 x nvox) with the zero-frequency rule of eq. 17:
// component c keeps (its average - target_c) when keep_c = 1 and drops its average when
// keep_c = 0.  out may alias A (A is read in full before out is written).
static void project_field(const GridPlan& g, bool fp32, bool plane, void* spec, const double* A,
                          const double* keep, const double* target, double* out, hipStream_t st) {
  if (plane) {
    PlaneArgs pa{PF_F64, A, spec};
    launch_plane_fwd(g, fp32, pa, nullptr, st);
  } else {
    XFwdArgs xf;
    std::memset(&xf, 0, sizeof(xf));
    xf.mode = XF_FIELD64;
    xf.in64 = A;
    xf.spec = spec;
    launch_xfwd(g, fp32, xf, st);
    launch_yfft(g, fp32, spec, -1, nullptr, st);
  }
  MidArgs m;
  std::memset(&m, 0, sizeof(m));
  m.op = MID_GREEN;
  m.spec = spec;
  for (int c = 0; c < 9; ++c) {
    m.mask_keep[c] = keep[c];
    m.dc_target[c] = target ? target[c] : 0.0;
  }
  m.inv_n = 1.0 / (double)g.nvox;
  launch_mid(g, fp32, m, st);
  if (plane) {
    PlaneInvArgs pi;
    std::memset(&pi, 0, sizeof(pi));
    pi.mode = PI_OUT64;
    pi.spec = spec;
    pi.out64 = out;
    launch_plane_inv(g, fp32, pi, st);
  } else {
    launch_yfft(g, fp32, spec, +1, nullptr, st);
    XInvArgs xi;
    std::memset(&xi, 0, sizeof(xi));
    xi.mode = XI_OUT64;
    xi.spec = spec;
    xi.out64 = out;
    launch_xinv(g, fp32, xi, st);
  }
}

// The Newton correction applied to F, in FP64.  FP64 form: the CG solution itself.  Mixed
// form: the FP32 CG solution carries components outside the range of G (its recurrences
// accumulate FP32 roundings over hundreds of iterations), and F would drift away from a
// compatible field; the correction is therefore widened to FP64 and projected again,
// G(x) with the same zero-frequency rule (F-controlled averages stay fixed), so that
// F - <F> stays a discrete gradient to FP64 rounding.
// The FP64 projection's plan and buffers (set up at rve_create for mixed handles).
static void prepare_correction(RVE& R) {
  if (R.proj_ready) return;
  build_plan(R.proj_plan, R.n, false, R.autotune, R.freq, R.stream);
  R.proj_spec.alloc(tsize(false) * 2 * 9 * R.proj_plan.g.nspec);
  R.x64.alloc(sizeof(double) * 9 * (size_t)R.nvox);
  R.proj_ready = true;
}

static const double* newton_correction(RVE& R, Work& w, const void* x, const double* keep) {
  if (!w.fp32) return static_cast<const double*>(x);
  prepare_correction(R);
  double* x64 = R.x64.as<double>();
  launch_widen(static_cast<const float*>(x), x64, 9 * R.nvox, R.stream);
  const GridPlan& g = R.proj_plan.g;
  project_field(g, false, plane_enabled() && plane_fits(g, false), R.proj_spec.p, x64, keep, nullptr, x64,
                R.stream);
  check_launch("newton correction");
  return x64;
}

// projected apply of a stress-like FP64 field: r = -G(P - Pbar), p = r, x = 0; returns r.r
static double run_residual(Ctx& C, RVE& R, Work& w, const double* P64, const double* mask_keep, const double* target,
                           void* x_zero) {
  const GridPlan& g = w.plan.g;
  if (w.plane) {
    PlaneArgs pa{PF_F64, P64, w.spec.p};
    {
      TimedLaunch t(R.tm(), KF_PLANE_FWD, bytes_plane_fwd_f64(g, w.fp32), R.stream);
      launch_plane_fwd(g, w.fp32, pa, nullptr, R.stream);
    }
    MidArgs m;
    std::memset(&m, 0, sizeof(m));
    m.op = MID_GREEN;
    m.spec = w.spec.p;
    for (int c = 0; c < 9; ++c) {
      m.mask_keep[c] = mask_keep[c];
      m.dc_target[c] = target ? target[c] : 0.0;
    }
    m.inv_n = 1.0 / (double)g.nvox;
    {
      TimedLaunch t(R.tm(), KF_MID, bytes_mid(g, w.fp32), R.stream);
      launch_mid(g, w.fp32, m, R.stream);
    }
    PlaneInvArgs pi;
    std::memset(&pi, 0, sizeof(pi));
    pi.mode = PI_RESID;
    pi.spec = w.spec.p;
    pi.x = x_zero;
    pi.r = w.r.p;
    pi.p = w.p.p;
    pi.partial = R.partial.as<double>();
    {
      TimedLaunch t(R.tm(), KF_PLANE_INV, bytes_plane_inv_resid(g, w.fp32), R.stream);
      launch_plane_inv(g, w.fp32, pi, R.stream);
    }
    launch_cg_start(R.cg.as<CGState>(), R.partial.as<double>(), plane_blocks(g), 0.0, 0, R.stream);
    check_launch("residual");
    HIPCHECK(hipMemcpyAsync(R.host_cg, R.cg.p, sizeof(CGState), hipMemcpyDeviceToHost, R.stream));
    HIPCHECK(hipStreamSynchronize(R.stream));
    R.timer.resolve();
    return R.host_cg->rr;
  }
  XFwdArgs xf;
  std::memset(&xf, 0, sizeof(xf));
  xf.mode = XF_FIELD64;
  xf.in64 = P64;
  xf.spec = w.spec.p;
  launch_xfwd(g, w.fp32, xf, R.stream);
  launch_yfft(g, w.fp32, w.spec.p, -1, nullptr, R.stream);
  MidArgs m;
  std::memset(&m, 0, sizeof(m));
  m.op = MID_GREEN;
  m.spec = w.spec.p;
  for (int c = 0; c < 9; ++c) {
    m.mask_keep[c] = mask_keep[c];
    m.dc_target[c] = target ? target[c] : 0.0;
  }
  m.inv_n = 1.0 / (double)g.nvox;
  launch_mid(g, w.fp32, m, R.stream);
  launch_yfft(g, w.fp32, w.spec.p, +1, nullptr, R.stream);
  XInvArgs xi;
  std::memset(&xi, 0, sizeof(xi));
  xi.mode = XI_RESID;
  xi.spec = w.spec.p;
  xi.x = x_zero;
  xi.r = w.r.p;
  xi.p = w.p.p;
  xi.partial = R.partial.as<double>();
  launch_xinv(g, w.fp32, xi, R.stream);
  launch_cg_start(R.cg.as<CGState>(), R.partial.as<double>(), xinv_blocks(g), 0.0, 0, R.stream);
  check_launch("residual");
  HIPCHECK(hipMemcpyAsync(R.host_cg, R.cg.p, sizeof(CGState), hipMemcpyDeviceToHost, R.stream));
  HIPCHECK(hipStreamSynchronize(R.stream));
  return R.host_cg->rr;
}

// conjugate gradients on G(K : x) = r (x, r, p set by run_residual); returns iterations
static int run_cg(Ctx& C, RVE& R, Work& w, void* x, const double* mask_keep, int& done_code,
                  bool transpose = false, double rr_floor = 0.0) {
  const GridPlan& g = w.plan.g;
  CGState* cg = R.cg.as<CGState>();
  double* part = R.partial.as<double>();
  const int nb = xfwd_blocks(g);
  // restart the CG bookkeeping from the residual just computed
  {
    CGState s = *R.host_cg;
    s.iter = 0;
    s.alpha = 0.0;
    s.rr_best = s.rr0;
    s.it_best = 0;
    s.done = (s.rr0 > 0.0 && C.opt.max_cg > 0) ? 0 : 1;
    s.tol2 = C.opt.cg_tol * C.opt.cg_tol;
    s.rr_floor = rr_floor;
    s.max_iter = C.opt.max_cg;
    s.stall = w.fp32 ? kCgStall : kCgStall64;
    *R.host_cg = s;
    HIPCHECK(hipMemcpyAsync(cg, R.host_cg, sizeof(CGState), hipMemcpyHostToDevice, R.stream));
  }
  XFwdArgs xf;
  std::memset(&xf, 0, sizeof(xf));
  xf.mode = XF_CG;
  xf.K = w.K.p;
  xf.gid = R.d_gid.as<int32_t>();
  xf.grainR = R.d_R.as<double>();
  xf.x = x;
  xf.xbest = w.xbest.p;
  xf.r = w.r.p;
  xf.p = w.p.p;
  xf.q = w.q.p;
  xf.cg = cg;
  xf.partial = part;
  xf.spec = w.spec.p;
  MidArgs m;
  std::memset(&m, 0, sizeof(m));
  m.op = MID_GREEN;
  m.spec = w.spec.p;
  for (int c = 0; c < 9; ++c) m.mask_keep[c] = mask_keep[c];
  m.inv_n = 1.0 / (double)g.nvox;
  m.cg = cg;
  XInvArgs xi;
  std::memset(&xi, 0, sizeof(xi));
  xi.mode = XI_CG;
  xi.spec = w.spec.p;
  xi.x = x;
  xi.r = w.r.p;
  xi.p = w.p.p;
  xi.q = w.q.p;
  xi.cg = cg;
  xi.partial = part;
  PrepArgs pr;
  std::memset(&pr, 0, sizeof(pr));
  pr.K = w.K.p;
  pr.gid = R.d_gid.as<int32_t>();
  pr.grainR = R.d_R.as<double>();
  pr.x = x;
  pr.xbest = w.xbest.p;
  pr.r = w.r.p;
  pr.p = w.p.p;
  pr.q = w.q.p;
  pr.y = w.y.p;
  pr.cg = cg;
  pr.partial = part;
  pr.k_scale = w.k16 ? R.mat.C11 : 1.0;
  PlaneArgs pa{PF_T, w.y.p, w.spec.p};
  pa.rr_partial = part;
  pa.n_rr = prep_blocks(g);
  PlaneInvArgs pi;
  std::memset(&pi, 0, sizeof(pi));
  pi.mode = PI_CG;
  pi.spec = w.spec.p;
  pi.x = x;
  pi.r = w.r.p;
  pi.p = w.p.p;
  pi.q = w.q.p;
  pi.cg = cg;
  pi.partial = part + 2048;
  // factorised projection (w.g3): partials of the stages in disjoint ranges of part:
  // [0, 1024) r.r of the prep, [3584, 3593) the zero-frequency term, [4096, 4096 + 9 nz)
  // plane sums of y, [16384, 16384 + kGradBlocks) p.q of the gradient pass (part holds at
  // least 12 x 2048 values)
  PlaneArgs pd{PF_DIV, w.y.p, w.spec.p};
  pd.rr_partial = part;
  pd.n_rr = prep_blocks(g);
  pd.plane_sums = part + 4096;
  MidArgs m3;
  std::memset(&m3, 0, sizeof(m3));
  m3.op = MID_GREEN3;
  m3.spec = w.spec.p;
  m3.inv_n = 1.0 / (double)g.nvox;
  m3.cg = cg;
  PlaneInvArgs pi3;
  std::memset(&pi3, 0, sizeof(pi3));
  pi3.mode = PI_OUT_T;
  pi3.spec = w.spec.p;
  pi3.cg = cg;
  pi3.out = w.w3.p;
  pi3.plane_sums = part + 4096;
  pi3.dc = part + 3584;
  for (int c = 0; c < 9; ++c) pi3.mask_keep[c] = mask_keep[c];
  pi3.inv_n = 1.0 / (double)g.nvox;
  GradArgs ga;
  std::memset(&ga, 0, sizeof(ga));
  ga.w = w.w3.p;
  ga.x = x;
  ga.dc = part + 3584;
  ga.r = w.r.p;
  ga.p = w.p.p;
  ga.q = w.q.p;
  ga.cg = cg;
  ga.partial = part + 16384;
  ga.lz = grad_lz(g);
  const int chunk = 4;
  int issued = 0;  // CG iterations launched so far
  auto issue_chunk = [&]() {
    for (int i = 0; i < chunk && w.plane; ++i, ++issued) {
      // the forward pass takes this iteration's beta step in its first block (no separate
      // launch); the alpha step, which every block of the next prep needs, has its own
      R.timer.tag = issued;
      pa.it = issued;
      {
        TimedLaunch t(R.tm(), KF_CG_PREP, bytes_cg_prep(g, w.fp32, w.k16, issued == 0), R.stream);
        launch_cg_prep(g, w.fp32, w.k16, transpose, pr, R.stream);
      }
      if (w.g3) {
        pd.it = issued;
        {
          TimedLaunch t(R.tm(), KF_PLANE_DIV, bytes_plane_div(g, w.fp32), R.stream);
          launch_plane_fwd(g, w.fp32, pd, cg, R.stream);
        }
        {
          TimedLaunch t(R.tm(), KF_MID3, bytes_mid3(g, w.fp32), R.stream);
          launch_mid(g, w.fp32, m3, R.stream);
        }
        {
          TimedLaunch t(R.tm(), KF_PLANE_W, bytes_plane_inv3(g, w.fp32), R.stream);
          launch_plane_inv(g, w.fp32, pi3, R.stream);
        }
        {
          TimedLaunch t(R.tm(), KF_CG_GRAD, bytes_cg_grad(g, w.fp32, issued == 0), R.stream);
          launch_cg_grad(g, w.fp32, ga, R.stream);
        }
        launch_cg_alpha(cg, part + 16384, grad_blocks(g, ga.lz), R.stream);
        continue;
      }
      {
        TimedLaunch t(R.tm(), KF_PLANE_FWD, bytes_plane_fwd_cg(g, w.fp32), R.stream);
        launch_plane_fwd(g, w.fp32, pa, cg, R.stream);
      }
      {
        TimedLaunch t(R.tm(), KF_MID, bytes_mid(g, w.fp32), R.stream);
        launch_mid(g, w.fp32, m, R.stream);
      }
      {
        TimedLaunch t(R.tm(), KF_PLANE_INV, bytes_plane_inv_cg(g, w.fp32, issued == 0), R.stream);
        launch_plane_inv(g, w.fp32, pi, R.stream);
      }
      launch_cg_alpha(cg, part + 2048, plane_blocks(g), R.stream);
    }
    R.timer.tag = -1;
    for (int i = 0; i < chunk && !w.plane; ++i) {
      launch_xfwd(g, w.fp32, xf, R.stream);
      launch_cg_beta(cg, part, nb, R.stream);
      launch_yfft(g, w.fp32, w.spec.p, -1, cg, R.stream);
      launch_mid(g, w.fp32, m, R.stream);
      launch_yfft(g, w.fp32, w.spec.p, +1, cg, R.stream);
      launch_xinv(g, w.fp32, xi, R.stream);
      launch_cg_alpha(cg, part, nb, R.stream);
    }
    check_launch("cg");
  };
  // snapshot of the CG scalars after the chunk just issued, into pinned slot s
  auto snapshot = [&](int s) {
    HIPCHECK(hipMemcpyAsync(&R.host_poll[s], cg, sizeof(CGState), hipMemcpyDeviceToHost, R.stream));
    HIPCHECK(hipEventRecord(R.poll_ev[s], R.stream));
  };
  // Chunks after the first differ from each other in nothing but the iteration tag (the
  // first iteration of a solve is the only special one), so with use_graph they are captured
  // once as a HIP graph per (transposed tangent, CG unknown) and replayed.
  const bool graph = C.use_graph && w.plane && !R.tm();
  auto issue_later_chunk = [&]() {
    if (!graph) {
      issue_chunk();
      return;
    }
    hipGraphExec_t& ge = w.cg_graph[transpose ? 1 : 0][x == w.xa.p ? 0 : 1];
    if (!ge) {
      hipGraph_t gr = nullptr;
      HIPCHECK(hipStreamBeginCapture(R.stream, hipStreamCaptureModeThreadLocal));
      issue_chunk();  // recorded, not run
      HIPCHECK(hipStreamEndCapture(R.stream, &gr));
      const hipError_t e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      HIPCHECK(e);
    } else {
      issued += chunk;
    }
    HIPCHECK(hipGraphLaunch(ge, R.stream));
  };
  if (!R.host_cg->done) {
    // the stop flag of chunk c - 1 is read while chunk c is already queued, so the GPU
    // never waits for the host; once the flag is set, the kernels of the chunk in flight
    // read it and return at once
    issue_chunk();
    snapshot(0);
    for (int c = 1;; ++c) {
      issue_later_chunk();
      snapshot(c & 1);
      HIPCHECK(hipEventSynchronize(R.poll_ev[(c - 1) & 1]));
      if (R.host_poll[(c - 1) & 1].done) break;
    }
  }
  // the last iteration's x += alpha p (its epilogue pass returned on the stop flag)
  launch_cg_finish(cg, w.fp32, x, w.p.p, 9 * g.nvox, R.stream);
  check_launch("cg finish");
  HIPCHECK(hipMemcpyAsync(R.host_cg, cg, sizeof(CGState), hipMemcpyDeviceToHost, R.stream));
  HIPCHECK(hipStreamSynchronize(R.stream));
  R.timer.resolve(R.host_cg->iter);
  done_code = R.host_cg->done;
  return R.host_cg->iter;
}

static double rms_of(Ctx& C, RVE& R, bool fp32, const void* f, int64_t n) {
  const int nb = launch_sumsq(f, fp32, n, R.partial.as<double>(), R.stream);
  std::vector<double> part(nb);
  HIPCHECK(hipMemcpyAsync(part.data(), R.partial.p, sizeof(double) * nb, hipMemcpyDeviceToHost, R.stream));
  HIPCHECK(hipStreamSynchronize(R.stream));
  double s = 0.0;
  for (double v : part) s += v;
  return std::sqrt(s / (double)n);
}

static void field_average(Ctx& C, RVE& R, const double* f, int ncomp, double* out) {
  const int nb = launch_colsum(f, ncomp, R.nvox, R.partial.as<double>(), R.stream);
  std::vector<double> part((size_t)nb * ncomp);
  HIPCHECK(hipMemcpyAsync(part.data(), R.partial.p, sizeof(double) * part.size(), hipMemcpyDeviceToHost, R.stream));
  HIPCHECK(hipStreamSynchronize(R.stream));
  for (int c = 0; c < ncomp; ++c) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(size_t)b * ncomp + c];
    out[c] = s / (double)R.nvox;
  }
}

static void run_nye(Ctx& C, RVE& R, Work& w) {
  const GridPlan& g = w.plan.g;
  if (w.plane) {
    PlaneArgs pa{PF_FPI, R.Fp.as<double>(), w.spec.p};
    launch_plane_fwd(g, w.fp32, pa, nullptr, R.stream);
    MidArgs m;
    std::memset(&m, 0, sizeof(m));
    m.op = MID_CURL;
    m.spec = w.spec.p;
    m.inv_n = 1.0 / (double)g.nvox;
    m.inv_h = 1.0 / R.h;
    launch_mid(g, w.fp32, m, R.stream);
    PlaneInvArgs pi;
    std::memset(&pi, 0, sizeof(pi));
    pi.mode = PI_OUT64;
    pi.spec = w.spec.p;
    pi.out64 = R.nye.as<double>();
    launch_plane_inv(g, w.fp32, pi, R.stream);
    launch_gnd(R.nvox, R.nye.as<double>(), R.d_gid.as<int32_t>(), R.d_R.as<double>(), R.d_mat.as<MatDev>(),
               R.rho_gnd.as<double>(), R.stream);
    check_launch("nye");
    return;
  }
  XFwdArgs xf;
  std::memset(&xf, 0, sizeof(xf));
  xf.mode = XF_FP_MINUS_I;
  xf.in64 = R.Fp.as<double>();
  xf.spec = w.spec.p;
  launch_xfwd(g, w.fp32, xf, R.stream);
  launch_yfft(g, w.fp32, w.spec.p, -1, nullptr, R.stream);
  MidArgs m;
  std::memset(&m, 0, sizeof(m));
  m.op = MID_CURL;
  m.spec = w.spec.p;
  m.inv_n = 1.0 / (double)g.nvox;
  m.inv_h = 1.0 / R.h;
  launch_mid(g, w.fp32, m, R.stream);
  launch_yfft(g, w.fp32, w.spec.p, +1, nullptr, R.stream);
  XInvArgs xi;
  std::memset(&xi, 0, sizeof(xi));
  xi.mode = XI_NYE;
  xi.spec = w.spec.p;
  xi.out64 = R.nye.as<double>();
  xi.rho_gnd = R.rho_gnd.as<double>();
  xi.gid = R.d_gid.as<int32_t>();
  xi.grainR = R.d_R.as<double>();
  xi.mat = R.d_mat.as<MatDev>();
  launch_xinv(g, w.fp32, xi, R.stream);
  check_launch("nye");
}

// Curl (eq. 12 with the rotated-scheme derivative) of a 9-component FP64 field on the FP64
// plane path: src is Fp (minus_identity: the curl of Fp - I) or a plain field.
static void curl_plane64(const GridPlan& g, void* spec, const double* src, bool minus_identity, double inv_h,
                         double* out, hipStream_t st) {
  PlaneArgs pa{minus_identity ? PF_FPI : PF_F64, src, spec};
  launch_plane_fwd(g, false, pa, nullptr, st);
  MidArgs m;
  std::memset(&m, 0, sizeof(m));
  m.op = MID_CURL;
  m.spec = spec;
  m.inv_n = 1.0 / (double)g.nvox;
  m.inv_h = inv_h;
  launch_mid(g, false, m, st);
  PlaneInvArgs pi;
  std::memset(&pi, 0, sizeof(pi));
  pi.mode = PI_OUT64;
  pi.spec = spec;
  pi.out64 = out;
  launch_plane_inv(g, false, pi, st);
}

// ------------------------------------------------------------------------------------
// one increment of one RVE (Section 2.2)
// ------------------------------------------------------------------------------------
// Newton iterations on G(P(F) - P_bar) = 0 from the field in R.F_work, with the average
// of the deformation-controlled components fixed by that field.  Returns RVE_OK when the
// applied correction falls below newton_tol; F_work then holds the solution and P_work,
// dg the matching stress and slip increments.
// Rounding floor of the mixed form's FP32 residual.  The projected residual G(P - P_bar) is
// formed from a stress field of magnitude rms(P) with FP32 transforms, so its rms carries a
// rounding error of about u32 rms(P) (u32 = 2^-24; measured: Newton stagnates at 1 to 2 times
// that value).  A conjugate-gradient solve stops once its residual is within kCgFloor of that
// floor (a smaller one is not resolved), and a Newton correction below newton_tol whose full
// step brings the residual within kNewtonFloor of it ends the increment even when CG did not
// converge: at the floor the right-hand side is rounding noise, to which the non-symmetric
// tangent can respond with a breakdown or a growing residual, and no FP32 correction can
// reduce the residual further.
// The FP64 form's floor is set by F itself: each entry of F carries a rounding error of about
// u64 (u64 = 2^-53, F of order one), which moves the stress by about C11 u64, far above the
// transforms' u64 rms(P) when the stress is small against the stiffness (measured on a cu64
// cell: Newton stagnates at 0.9 to 1.1 times u64 C11).  Its floor is u64 times the rms over the
// voxels of their C11.  That estimate is only an upper bound where stiff phases are a small
// part of the cell (a 1e6 stiffness-contrast cell converged to a fifth of it), so in FP64 it
// does not stop CG; it only lets a Newton correction below newton_tol whose full step brings the
// residual within kNewtonFloor64 of it end the increment after a CG that did not converge.
constexpr double kU32 = 5.9604644775390625e-08;
constexpr double kU64 = 1.1102230246251565e-16;
constexpr double kCgFloor = 8.0;
constexpr double kNewtonFloor = 32.0;
constexpr double kNewtonFloor64 = 4.0;

static int32_t newton_solve(Ctx& C, RVE& R, Work& w, const double* keep, const double* Pbar, double dt, rve_step_stats& st,
                            const char** why) {
  const int64_t nv = R.nvox;
  const double n9 = 9.0 * (double)nv;
  // rounding floor of the residual: u32 rms(P) at the current iterate (mixed form), u64 rms(C11)
  double p_floor = w.fp32 ? 0.0 : kU64 * R.c11_rms;
  auto update_floor = [&]() {
    if (w.fp32) p_floor = kU32 * rms_of(C, R, false, R.P_work.as<double>(), 9 * nv);
  };
  LocalStats ls = run_constitutive(C, R, w, R.F_work.as<double>(), nullptr, 0.0, nullptr, dt, true);
  st.local_iters_max = std::max(st.local_iters_max, ls.max_iters);
  if (ls.failures) {
    *why = "local Newton did not converge at the initial guess";
    return RVE_ENOCONV;
  }
  void* x = w.xa.p;     // CG unknown of the current Newton step
  void* xo = w.xb.p;    // the other one
  double rr = run_residual(C, R, w, R.P_work.as<double>(), keep, Pbar, x);
  st.residual_evals++;
  double res = std::sqrt(rr / n9);
  if (!std::isfinite(res)) {
    *why = "non-finite residual at the initial guess";
    return RVE_ENOCONV;
  }
  update_floor();
  for (int it = 0; it < C.opt.max_newton; ++it) {
    int done = 0;
    const double cg_floor = w.fp32 ? kCgFloor * p_floor : 0.0;
    const int ncg = run_cg(C, R, w, x, keep, done, false, cg_floor * cg_floor * n9);
    const CGState cg_end = *R.host_cg;
    st.cg_iters += ncg;
    // A breakdown (negative curvature along p), a diverging or stalled residual or the
    // iteration cap ends CG early, as in truncated CG.  The correction is then the iterate
    // with the smallest r.r seen, if any iterate improved on the start (the current one
    // unless r.r has grown since; after a converged solve the current r.r is the smallest),
    // and the residual line search below decides whether it is usable.  Only a solve that
    // converged, or stalled at its rounding floor, can end the Newton iteration: a small
    // correction from a broken-down solve says nothing about the residual.
    const bool cg_ok = done == 1 || done == 5;
    const bool use_best = done != 1 && cg_end.it_best > 0 && cg_end.rr > cg_end.rr_best;
    const double* corr = newton_correction(R, w, use_best ? w.xbest.p : x, keep);
    const double dF = rms_of(C, R, false, corr, 9 * nv);
    if (!std::isfinite(dF)) {
      *why = "non-finite Newton correction";
      return RVE_ENOCONV;
    }
    st.newton_iters++;
    double lam = 1.0, res_try = 0.0, lam_base = 0.0;
    bool accepted = false, at_floor = false;
    for (int ls_i = 0; ls_i <= C.opt.max_backtrack; ++ls_i) {
      LocalStats l2 = run_constitutive(C, R, w, R.F_work.as<double>(), corr, lam, R.F_try.as<double>(), dt, true,
                                       true, lam_base);
      lam_base = lam;
      st.local_iters_max = std::max(st.local_iters_max, l2.max_iters);
      if (l2.failures == 0) {
        const double rr_t = run_residual(C, R, w, R.P_work.as<double>(), keep, Pbar, xo);
        st.residual_evals++;
        res_try = std::sqrt(rr_t / n9);
        at_floor = lam == 1.0 && dF <= C.opt.newton_tol && res_try <= (w.fp32 ? kNewtonFloor : kNewtonFloor64) * p_floor;
        // a full correction below the tolerance is applied without a decrease test (the
        // residual is then at its rounding floor); otherwise the residual must not grow
        if (std::isfinite(res_try) &&
            (res_try <= res || (lam == 1.0 && dF <= C.opt.newton_tol && cg_ok) || at_floor)) {
          accepted = true;
          break;
        }
      }
      lam *= 0.5;
      st.line_search_cuts++;
    }
    if (trace_on())
      std::fprintf(stderr,
                   "[rve] newton %d: cg %d (code %d, rr/rr0 %.2e%s) |dF| %.3e lam %.4g res %.4e -> %.4e%s%s local_it %d "
                   "floor %.3e\n",
                   it + 1, ncg, done, cg_end.rr / cg_end.rr0, use_best ? ", best iterate" : "", dF, lam, res, res_try,
                   accepted ? "" : " (line search failed)", at_floor ? " (at the rounding floor)" : "",
                   st.local_iters_max, p_floor);
    if (!accepted) {
      *why = "residual line search failed";
      return RVE_ENOCONV;
    }
    std::swap(R.F_work.p, R.F_try.p);
    std::swap(x, xo);
    res = res_try;
    st.dF_norm = dF;
    st.res_norm = res;
    // converged when the full Newton correction (not a line-search fraction of it) of a
    // usable linear solve is small, or (mixed form) when such a correction has brought the
    // residual to its FP32 rounding floor
    if (lam == 1.0 && dF <= C.opt.newton_tol && (cg_ok || at_floor)) return RVE_OK;
    update_floor();
  }
  *why = "Newton did not converge within max_newton";
  return RVE_ENOCONV;
}

// Increment k.  The initial guess extrapolates the previous field increment, with the
// average of the deformation-controlled components set to the target.  If Newton fails
// from there, the same increment (same dt, same start-of-increment state) is solved again
// by continuation in the load: targets F_bar(s) = F_bar_{k-1} + s (F_bar_k - F_bar_{k-1})
// for s = 1/m, 2/m, ..., 1 (m = 2, 4, 8, 16), each solve started from the previous root.
// Only the s = 1 problem is the increment, so the committed solution is the same.
static int32_t step_rve(Ctx& C, RVE& R, const double* Fbar, const uint8_t* mask, const double* Pbar, double dt,
                        rve_step_stats& st) {
  std::memset(&st, 0, sizeof(st));
  const int64_t nv = R.nvox;
  double keep[9];
  for (int c = 0; c < 9; ++c) keep[c] = mask[c] ? 0.0 : 1.0;
  HIPCHECK(hipMemcpyAsync(R.dg_saved.p, R.dg.p, sizeof(double) * 12 * nv, hipMemcpyDeviceToDevice, R.stream));
  auto restore_dg = [&]() {
    HIPCHECK(hipMemcpyAsync(R.dg.p, R.dg_saved.p, sizeof(double) * 12 * nv, hipMemcpyDeviceToDevice, R.stream));
  };
  const char* why = "";
  int64_t discarded = 0;  // projected applies of failed attempts (not part of the committed solve)
  auto attempt = [&](Work& w, int max_stages) -> int32_t {
    // direct attempt
    Corr9 cr;
    for (int c = 0; c < 9; ++c) {
      const double dmac = mask[c] ? (Fbar[c] - R.Fbar_prev[c]) : 0.0;
      const double dprev = R.have_prev ? (R.Favg[c] - R.Favg_prev[c]) : 0.0;
      cr.v[c] = mask[c] ? (dmac - dprev) : 0.0;
    }
    launch_predictor(R.F.as<double>(), R.have_prev ? R.F_prev.as<double>() : nullptr, cr, R.F_work.as<double>(),
                     nv, R.stream);
    check_launch("predictor");
    int32_t rc = newton_solve(C, R, w, keep, Pbar, dt, st, &why);
    st.continuation_stages = 0;
    for (int m = 2; rc != RVE_OK && m <= max_stages; m *= 2) {
      if (trace_on()) std::fprintf(stderr, "[rve] %s; load continuation with %d stages\n", why, m);
      discarded = (int64_t)st.residual_evals + st.cg_iters;  // the failed solve is not the increment's
      st.continuation_stages = m;
      restore_dg();
      Corr9 zero;
      for (int c = 0; c < 9; ++c) zero.v[c] = 0.0;
      launch_predictor(R.F.as<double>(), nullptr, zero, R.F_work.as<double>(), nv, R.stream);
      double Fb_prev[9];
      std::memcpy(Fb_prev, R.Fbar_prev, sizeof(Fb_prev));
      rc = RVE_OK;
      for (int sidx = 1; sidx <= m && rc == RVE_OK; ++sidx) {
        const double s = (double)sidx / (double)m;
        Corr9 step;
        for (int c = 0; c < 9; ++c) {
          const double target = R.Fbar_prev[c] + s * (Fbar[c] - R.Fbar_prev[c]);
          step.v[c] = mask[c] ? (target - Fb_prev[c]) : 0.0;
          Fb_prev[c] = target;
        }
        launch_predictor(R.F_work.as<double>(), nullptr, step, R.F_work.as<double>(), nv, R.stream);
        check_launch("predictor");
        rc = newton_solve(C, R, w, keep, Pbar, dt, st, &why);
      }
    }
    return rc;
  };
  // FP32: one direct attempt, then the FP64 path with load continuation
  int32_t rc = attempt(work(R, C.fp32), C.fp32 ? 1 : C.max_continuation);
  if (rc != RVE_OK && C.fp32) {
    // FP32 conjugate gradients stall near kappa * eps_32 on ill-conditioned tangents;
    // solve this increment with the FP64 spectral path instead.
    if (trace_on()) std::fprintf(stderr, "[rve] %s in FP32; increment solved again in FP64\n", why);
    restore_dg();
    discarded = (int64_t)st.residual_evals + st.cg_iters;
    st.fp64_fallback = 1;
    R.fp64_fallbacks++;
    rc = attempt(work(R, false), C.max_continuation);
  }
  if (rc != RVE_OK) {
    restore_dg();
    // the tangents now belong to a failed iterate, not to the last converged increment
    R.w[0].k_ready = R.w[1].k_ready = false;
    HIPCHECK(hipStreamSynchronize(R.stream));
    st.status = rc;
    g_last_error = why;
    return rc;
  }
  // keep the start-of-increment state (the reverse pass of this increment needs it)
  HIPCHECK(hipMemcpyAsync(R.Fp_prev.p, R.Fp.p, sizeof(double) * 9 * nv, hipMemcpyDeviceToDevice, R.stream));
  HIPCHECK(hipMemcpyAsync(R.rho_ssd_prev.p, R.rho_ssd.p, sizeof(double) * 12 * nv, hipMemcpyDeviceToDevice, R.stream));
  HIPCHECK(hipMemcpyAsync(R.rho_gnd_prev.p, R.rho_gnd.p, sizeof(double) * 12 * nv, hipMemcpyDeviceToDevice, R.stream));
  R.dt_last = dt;
  // commit: Fp and rho_SSD from the converged slip increments, then the Nye tensor
  CommitArgs ca;
  ca.nvox = nv;
  ca.gid = R.d_gid.as<int32_t>();
  ca.grainR = R.d_R.as<double>();
  ca.mat = R.d_mat.as<MatDev>();
  ca.dg = R.dg.as<double>();
  ca.Fp = R.Fp.as<double>();
  ca.rho_ssd = R.rho_ssd.as<double>();
  ca.rho_gnd = R.rho_gnd.as<double>();
  launch_commit(ca, R.stream);
  check_launch("commit");
  std::swap(R.F_prev.p, R.F.p);     // F_prev <- F_{k-1}
  std::swap(R.F.p, R.F_work.p);     // F <- F_k
  std::swap(R.P.p, R.P_work.p);
  run_nye(C, R, work(R, C.fp32));
  std::memcpy(R.Favg_prev, R.Favg, sizeof(R.Favg));
  field_average(C, R, R.F.as<double>(), 9, R.Favg);
  field_average(C, R, R.P.as<double>(), 9, R.Pavg);
  std::memcpy(R.Fbar_prev, Fbar, sizeof(double) * 9);
  std::memcpy(R.Pbar_prev, Pbar, sizeof(double) * 9);
  R.have_prev = true;
  R.increments++;
  st.status = RVE_OK;
  // the metric counts the projected applies of the solve that produced the committed
  // increment; those of failed attempts before it are reported separately
  st.voxel_iterations = (double)nv * (double)((int64_t)st.residual_evals + st.cg_iters - discarded);
  st.discarded_voxel_iterations = (double)nv * (double)discarded;
  return RVE_OK;
}

// Automatic time-step cut-back: an increment that fails (after the solver's own retries) is
// replaced by two increments of half the time step, to the midpoint of the macroscopic
// targets (both the prescribed F and the prescribed P interpolate linearly in time) and then
// to the end point, each committed like any increment; a half that fails is halved again,
// down to max_cutbacks levels.  Unlike the load continuation inside step_rve (which changes
// only the iteration path of one increment), a cut-back changes the time integration: the
// state is committed at the midpoint, so the result equals that of two explicit increments.
// st accumulates the counts of every attempt; st.cutbacks counts the halvings.
static int32_t step_with_cutback(Ctx& C, RVE& R, const double* Fbar, const uint8_t* mask, const double* Pbar, double dt,
                                 int depth, rve_step_stats& st) {
  rve_step_stats s1;
  const int32_t rc = step_rve(C, R, Fbar, mask, Pbar, dt, s1);
  auto add = [&](const rve_step_stats& a) {
    st.newton_iters += a.newton_iters;
    st.cg_iters += a.cg_iters;
    st.residual_evals += a.residual_evals;
    st.line_search_cuts += a.line_search_cuts;
    st.local_iters_max = std::max(st.local_iters_max, a.local_iters_max);
    st.res_norm = a.res_norm;
    st.dF_norm = a.dF_norm;
    st.fp64_fallback |= a.fp64_fallback;
    st.continuation_stages = std::max(st.continuation_stages, a.continuation_stages);
    if (a.status == RVE_OK) {
      st.voxel_iterations += a.voxel_iterations;
      st.discarded_voxel_iterations += a.discarded_voxel_iterations;
    } else {
      // every projected apply of a failed attempt is discarded
      st.discarded_voxel_iterations += (double)R.nvox * (double)(a.residual_evals + a.cg_iters);
    }
  };
  add(s1);
  if (rc == RVE_OK || rc != RVE_ENOCONV || depth >= C.max_cutbacks) {
    st.status = rc;
    return rc;
  }
  if (trace_on()) std::fprintf(stderr, "[rve] increment failed; time step cut back to dt / %d\n", 2 << depth);
  st.cutbacks += 1;
  double Fm[9], Pm[9];
  for (int c = 0; c < 9; ++c) {
    Fm[c] = 0.5 * (R.Fbar_prev[c] + Fbar[c]);
    Pm[c] = 0.5 * (R.Pbar_prev[c] + Pbar[c]);
  }
  int32_t r = step_with_cutback(C, R, Fm, mask, Pm, 0.5 * dt, depth + 1, st);
  if (r == RVE_OK) r = step_with_cutback(C, R, Fbar, mask, Pbar, 0.5 * dt, depth + 1, st);
  st.status = r;
  return r;
}

}  // namespace rve

// ======================================================================================
// C ABI
// ======================================================================================
using namespace rve;

struct rve_ctx : Ctx {};

template <typename Fn>
static int32_t guarded(Fn fn) {
  try {
    g_last_error.clear();
    return fn();
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return RVE_EDEVICE;
  }
}

// Raise the dynamic-LDS limit of the LDS-staged kernels to what the current device
// allows, once per device, before any launch on it: changing a kernel attribute while
// other threads launch that kernel is not safe.  Best effort: a launch that asks for more
// LDS than the device grants fails and is reported by the launch check that follows it.
static void prepare_device() {
  static std::mutex mu;
  static std::vector<int> done;
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if (std::find(done.begin(), done.end(), dev) != done.end()) return;
  int lds = 0;
  HIPCHECK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const hipError_t e1 = set_spectral_lds_limits(lds), e2 = set_plane_lds_limits(lds);
  if ((e1 != hipSuccess || e2 != hipSuccess) && trace_on())
    std::fprintf(stderr, "[rve] dynamic LDS limit not raised: %s\n", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  (void)hipGetLastError();
  done.push_back(dev);
}

// ------------------------------------------------------------------------------------
// Projection without allocation (rve_project_noalloc)
// ------------------------------------------------------------------------------------
// Working memory of rve_project_noalloc: the half spectrum and the root tables, in one fixed
// device array (each device holds its own copy until the process ends).  Host code never
// passes the array's name to a kernel or a copy: it takes the device address once per device
// from hipGetSymbolAddress (noalloc_base) and uses that.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr size_t kNoAllocTables = size_t(64) << 10;  // 3 axes x (tw, E) x 256 roots x 16 B = 24 KiB
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static void* noalloc_base() {
  static std::mutex mu;
  static std::vector<std::pair<int, void*>> addr;  // (device, address of scratch there)
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  for (const auto& e : addr)
    if (e.first == dev) return e.second;
  void* p = nullptr;
  HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error(RVE_EDEVICE, "no device address for the projection scratch array");
  addr.emplace_back(dev, p);
  return p;
}

// Root tables of one axis of length n on the device: tw[k] = exp(-2 pi i k / n) in the
// spectral precision T, E[q] = exp(+2 pi i q / n) in FP64, exact at the quarter turns.
template <typename T>
__global__ void k_root_tables(int n, T* tw, double* E) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s, c;
  sincospi(2.0 * (double)k / (double)n, &s, &c);
  if (k == 0) { c = 1.0; s = 0.0; }
  if (2 * k == n) { c = -1.0; s = 0.0; }
  if (4 * k == n) { c = 0.0; s = 1.0; }
  if (4 * k == 3 * n) { c = 0.0; s = -1.0; }
  tw[2 * k] = (T)c;
  tw[2 * k + 1] = (T)(-s);
  E[2 * k] = c;
  E[2 * k + 1] = s;
}

// The grid plan of rve_project_noalloc inside the scratch array: tables at base, the
// spectrum from base + kNoAllocTables.  Throws RVE_EINVAL (before touching the device when
// base is null) if the grid does not fit.
static void noalloc_plan(GridPlan& g, const int n[3], bool fp32, unsigned char* base, void** spec) {
  plan_geometry(g, n);
  const size_t spec_bytes = tsize(fp32) * 2 * 9 * (size_t)g.nspec;
  if (spec_bytes > kNoAllocBytes - kNoAllocTables)
    throw Error(RVE_EINVAL, "grid too large for rve_project_noalloc: its spectrum needs " +
                                std::to_string(spec_bytes) + " bytes, the scratch array holds " +
                                std::to_string(kNoAllocBytes - kNoAllocTables));
  if (!base) return;
  const void** tw[3] = {&g.twx, &g.twy, &g.twz};
  const void** E[3] = {&g.Ex, &g.Ey, &g.Ez};
  for (int d = 0; d < 3; ++d) {
    *tw[d] = base + (size_t)d * 8192;             // 256 roots x 16 B at most
    *E[d] = base + (size_t)(3 + d) * 8192;
  }
  *spec = base + kNoAllocTables;
}

// The autotuner: for a grid size and spectral precision, time the z pass (z transforms and
// the projection of eq. 17) at each candidate tile width (kx columns per block: the widest
// that the 256-thread block holds, then halvings down to 1) and keep the fastest for the
// process; the same for the three-component z pass of the factorised projection.  The tile
// width changes the work split, not the arithmetic of any line or frequency, so the choice
// does not change results.  Runs once per (grid, precision), on the creating thread, before
// any worker exists.
static void autotune_grid(const int32_t n_in[3], bool fp32) {
  const int n[3] = {n_in[0], n_in[1], n_in[2]};
  if (tuned_tz(n, fp32).tz > 0) return;
  Plan P;
  build_plan(P, n, fp32, false);
  const GridPlan base = P.g;
  TunedTiles best;
  best.tz = base.tz;
  best.tz3 = base.tz3;
  DevBuf spec;
  spec.alloc(tsize(fp32) * 2 * 9 * (size_t)base.nspec);
  HIPCHECK(hipMemset(spec.p, 0, spec.bytes));
  hipStream_t st = nullptr;
  HIPCHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  MidArgs m;
  std::memset(&m, 0, sizeof(m));
  m.spec = spec.p;
  m.inv_n = 1.0 / (double)base.nvox;
  // fastest of the candidate widths (first = widest) for one operator
  auto tune = [&](int op, int widest) {
    std::vector<int> cand;
    for (int t = widest; t >= 1; t /= 2) cand.push_back(t);
    m.op = op;
    int pick = cand.front();
    float best_ms = 1e30f;
    for (int t : cand) {
      GridPlan g = base;
      if (op == MID_GREEN3) {
        g.tz3 = t;
        g.ftz3 = make_fastdiv(t);
      } else {
        g.tz = t;
        g.ftz = make_fastdiv(t);
      }
      launch_mid(g, fp32, m, st);  // warm-up
      HIPCHECK(hipEventRecord(e0, st));
      for (int r = 0; r < 5; ++r) launch_mid(g, fp32, m, st);
      HIPCHECK(hipEventRecord(e1, st));
      HIPCHECK(hipEventSynchronize(e1));
      check_launch("autotune");
      float ms = 0.f;
      HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
      if (trace_on())
        std::fprintf(stderr, "[rve] autotune %dx%dx%d %s %s: tz %d %.2f us\n", n[0], n[1], n[2], fp32 ? "fp32" : "fp64",
                     op == MID_GREEN3 ? "3-comp" : "9-comp", t, 1e3f * ms / 5.f);
      if (ms < best_ms) best_ms = ms, pick = t;
    }
    return pick;
  };
  best.tz = tune(MID_GREEN, base.tz);
  if (factorised_fits(base)) best.tz3 = tune(MID_GREEN3, std::max(1, std::min(base.nxh, 768 / base.nz)));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tuned_tz.push_back({TuneKey{n[0], n[1], n[2], fp32 ? 1 : 0}, best});
}

extern "C" {

int32_t rve_create(const rve_desc* descs, int32_t n_rve, const rve_options* opt, rve_handle* out) {
  return guarded([&]() -> int32_t {
    if (!descs || n_rve < 1 || !out) throw Error(RVE_EINVAL, "need descs, n_rve >= 1 and out");
    std::unique_ptr<rve_ctx> C(new rve_ctx());
    rve_options o;
    std::memset(&o, 0, sizeof(o));
    o.precision = RVE_FP64;
    o.newton_tol = 1e-10;
    o.cg_tol = 1e-8;
    o.max_newton = 40;
    o.max_cg = 2000;
    o.max_backtrack = 12;
    if (opt) o = *opt;
    if (o.precision != RVE_FP64 && o.precision != RVE_MIXED) throw Error(RVE_EINVAL, "unknown precision");
    if (!(o.newton_tol > 0) || !(o.cg_tol > 0) || o.max_newton < 1 || o.max_cg < 1 || o.max_backtrack < 0)
      throw Error(RVE_EINVAL, "bad solver options");
    C->opt = o;
    C->fp32 = o.precision == RVE_MIXED;
    C->device = o.device;
    HIPCHECK(hipSetDevice(C->device));
    prepare_device();
    C->stream = (hipStream_t)o.stream;
    C->workers = o.workers > 0 ? o.workers : settings().workers;
    C->use_graph = o.use_graph != 0;
    if (o.max_cutbacks < 0 || o.max_cutbacks > 10 || o.max_continuation < 0) throw Error(RVE_EINVAL, "bad solver options");
    C->max_cutbacks = o.max_cutbacks;
    if (o.frequencies != FREQ_ROTATED && o.frequencies != FREQ_STANDARD) throw Error(RVE_EINVAL, "unknown frequency scheme");
    C->freq = o.frequencies;
    if (o.projection != 0 && o.projection != 1) throw Error(RVE_EINVAL, "unknown projection form");
    C->factorised = o.projection == 0;
    C->max_continuation = o.max_continuation > 0 ? o.max_continuation : 16;
    C->autotune = o.autotune != 0;
    if (C->autotune)
      for (int i = 0; i < n_rve; ++i) {
        autotune_grid(descs[i].n, C->fp32);
        if (C->fp32) autotune_grid(descs[i].n, false);  // FP64 projection of the correction
      }
    for (int i = 0; i < n_rve; ++i) {
      C->rves.emplace_back(new RVE());
      init_rve(*C, *C->rves.back(), descs[i]);
    }
    *out = C.release();
    return RVE_OK;
  });
}

int32_t rve_timing_start(rve_handle h, uint32_t mask) {
  return guarded([&]() -> int32_t {
    if (!h) throw Error(RVE_EINVAL, "null handle");
    if (mask >> KF_COUNT) throw Error(RVE_EINVAL, "unknown kernel family in mask");
    HIPCHECK(hipSetDevice(h->device));
    for (auto& R : h->rves) {
      HIPCHECK(hipStreamSynchronize(R->stream));
      R->timer.resolve();
      R->timer.reset(mask);
    }
    return RVE_OK;
  });
}

int32_t rve_timing_read(rve_handle h, int32_t family, int64_t* launches, double* total_ms, double* units) {
  return guarded([&]() -> int32_t {
    if (!h) throw Error(RVE_EINVAL, "null handle");
    if (family < 0 || family >= KF_COUNT) throw Error(RVE_EINVAL, "unknown kernel family");
    int64_t n = 0;
    double t = 0.0, u = 0.0;
    for (auto& R : h->rves) {
      n += R->timer.launches[family];
      t += R->timer.ms[family];
      u += R->timer.bytes[family];
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = t;
    if (units) *units = u;
    return RVE_OK;
  });
}

void rve_destroy(rve_handle h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  for (auto& r : h->rves) (void)hipStreamSynchronize(r->stream);
  h->rves.clear();
  delete h;
}

const char* rve_last_error(void) { return g_last_error.c_str(); }

int32_t rve_step_increment(rve_handle h, const double* F_bar, const uint8_t* mask, const double* P_bar, double dt,
                           rve_step_stats* stats) {
  return guarded([&]() -> int32_t {
    if (!h || !F_bar || !mask) throw Error(RVE_EINVAL, "null argument");
    if (!(std::isfinite(dt) && dt > 0)) throw Error(RVE_EINVAL, "dt must be > 0");
    const int nr = (int)h->rves.size();
    for (int i = 0; i < 9 * nr; ++i)
      if (!std::isfinite(F_bar[i]) || (P_bar && !std::isfinite(P_bar[i])))
        throw Error(RVE_EINVAL, "non-finite load target");
    HIPCHECK(hipSetDevice(h->device));
    std::vector<double> zeros(9 * (size_t)nr, 0.0);
    const double* Pb = P_bar ? P_bar : zeros.data();
    // work queued on the caller's stream comes first
    if (h->stream) {
      hipEvent_t ev;
      HIPCHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      HIPCHECK(hipEventRecord(ev, h->stream));
      for (auto& r : h->rves) HIPCHECK(hipStreamWaitEvent(r->stream, ev, 0));
      HIPCHECK(hipEventDestroy(ev));
    }
    // RVEs are independent: host workers drive them concurrently, one stream each, so
    // that small grids share the GPU (the host loop of one RVE synchronises on its own
    // stream only).
    std::vector<rve_step_stats> st(nr);
    std::vector<int32_t> rcs(nr, RVE_OK);
    std::vector<std::string> msgs(nr);
    // the workers take the RVEs in the handle's order (on the mixed-size sweep this beat
    // longest-first, shortest-first and alternating orders: a tail of small RVEs alone leaves
    // the GPU idle, and a block of large ones at the start does too little with the rest)
    std::atomic<int> next(0);
    auto worker = [&]() {
      (void)hipSetDevice(h->device);
      for (;;) {
        const int i = next.fetch_add(1);
        if (i >= nr) break;
        try {
          if (h->max_cutbacks > 0) {
            std::memset(&st[i], 0, sizeof(st[i]));
            rcs[i] = step_with_cutback(*h, *h->rves[i], F_bar + 9 * i, mask, Pb + 9 * i, dt, 0, st[i]);
          } else {
            rcs[i] = step_rve(*h, *h->rves[i], F_bar + 9 * i, mask, Pb + 9 * i, dt, st[i]);
          }
          if (rcs[i] != RVE_OK) msgs[i] = g_last_error;
        } catch (const Error& e) {
          rcs[i] = e.code;
          msgs[i] = e.what();
          st[i].status = e.code;
        } catch (const std::exception& e) {
          rcs[i] = RVE_EDEVICE;
          msgs[i] = e.what();
          st[i].status = RVE_EDEVICE;
        }
      }
    };
    const int nw = std::max(1, std::min(nr, h->workers));
    if (nw == 1) {
      worker();
    } else {
      std::vector<std::thread> pool;
      for (int t = 0; t < nw; ++t) pool.emplace_back(worker);
      for (auto& t : pool) t.join();
    }
    if (stats)
      for (int i = 0; i < nr; ++i) stats[i] = st[i];
    int32_t worst = RVE_OK;
    std::string msg;
    for (int i = 0; i < nr; ++i)
      if (rcs[i] != RVE_OK) {
        worst = rcs[i];
        msg = "rve " + std::to_string(i) + ": " + msgs[i];
      }
    if (worst != RVE_OK) throw Error(worst, msg);
    return RVE_OK;
  });
}

int32_t rve_macro_stress(rve_handle h, int32_t rve, double* P_avg, double* F_avg, double* sigma) {
  return guarded([&]() -> int32_t {
    if (!h || rve < 0 || rve >= (int32_t)h->rves.size()) throw Error(RVE_EINVAL, "bad rve index");
    const RVE& R = *h->rves[rve];
    if (P_avg) std::memcpy(P_avg, R.Pavg, sizeof(double) * 9);
    if (F_avg) std::memcpy(F_avg, R.Favg, sizeof(double) * 9);
    if (sigma) {
      const double* F = R.Favg;
      const double det = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
                         F[2] * (F[3] * F[7] - F[4] * F[6]);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double s = 0.0;
          for (int k = 0; k < 3; ++k) s += R.Pavg[3 * i + k] * F[3 * j + k];
          sigma[3 * i + j] = s / det;
        }
    }
    return RVE_OK;
  });
}

int32_t rve_get_field(rve_handle h, int32_t rve, int32_t which, double* out) {
  return guarded([&]() -> int32_t {
    if (!h || rve < 0 || rve >= (int32_t)h->rves.size() || !out) throw Error(RVE_EINVAL, "bad argument");
    RVE& R = *h->rves[rve];
    const DevBuf* b = nullptr;
    int nc = 9;
    switch (which) {
      case 0: b = &R.F; break;
      case 1: b = &R.P; break;
      case 2: b = &R.Fp; break;
      case 3: b = &R.rho_ssd; nc = 12; break;
      case 4: b = &R.rho_gnd; nc = 12; break;
      case 5: b = &R.nye; break;
      case 6: b = &R.dg; nc = 12; break;
      default: throw Error(RVE_EINVAL, "unknown field");
    }
    HIPCHECK(hipSetDevice(h->device));
    HIPCHECK(hipMemcpyAsync(out, b->p, sizeof(double) * nc * R.nvox, hipMemcpyDeviceToHost, R.stream));
    HIPCHECK(hipStreamSynchronize(R.stream));
    return RVE_OK;
  });
}

int32_t rve_nye_gnd(rve_handle h, int32_t rve, double* nye, double* rho_gnd) {
  return guarded([&]() -> int32_t {
    if (!h || rve < 0 || rve >= (int32_t)h->rves.size()) throw Error(RVE_EINVAL, "bad rve index");
    int32_t rc = RVE_OK;
    if (nye) rc = rve_get_field(h, rve, 5, nye);
    if (rc == RVE_OK && rho_gnd) rc = rve_get_field(h, rve, 4, rho_gnd);
    return rc;
  });
}

int32_t rve_adjoint_solve(rve_handle h, int32_t rve, const uint8_t* mask, const double* g, double* lambda,
                          int32_t* cg_iters) {
  return guarded([&]() -> int32_t {
    if (!h || rve < 0 || rve >= (int32_t)h->rves.size() || !mask || !g || !lambda)
      throw Error(RVE_EINVAL, "bad argument");
    if (h->fp32) throw Error(RVE_EINVAL, "the adjoint solve needs an RVE_FP64 handle");
    HIPCHECK(hipSetDevice(h->device));
    RVE& R = *h->rves[rve];
    Work& w = work(R, false);
    if (!w.k_ready) throw Error(RVE_EINVAL, "no tangent yet: take an increment first");
    if (!w.plane) throw Error(RVE_EINVAL, "the adjoint solve needs the plane kernels");
    double keep[9];
    for (int c = 0; c < 9; ++c) keep[c] = mask[c] ? 0.0 : 1.0;
    // r = -G(g), x = 0; CG on G(K^T : x) = r gives x = -lambda
    void* x = w.xa.p;
    run_residual(*h, R, w, g, keep, nullptr, x);
    int done = 0;
    const int n = run_cg(*h, R, w, x, keep, done, true);
    launch_negate(static_cast<const double*>(x), lambda, 9 * R.nvox, R.stream);
    check_launch("adjoint");
    HIPCHECK(hipStreamSynchronize(R.stream));
    if (cg_iters) *cg_iters = n;
    return (done == 1 || done == 5) ? RVE_OK : RVE_ENOCONV;
  });
}

int32_t rve_adjoint_increment(rve_handle h, int32_t rve, const uint8_t* mask, const double* dLdP, double* Fp_bar,
                              double* rho_bar, double* theta_bar, int32_t* cg_iters) {
  return guarded([&]() -> int32_t {
    if (!h || rve < 0 || rve >= (int32_t)h->rves.size() || !mask || !dLdP || !Fp_bar || !rho_bar || !theta_bar)
      throw Error(RVE_EINVAL, "bad argument");
    for (int i = 0; i < 9; ++i)
      if (!std::isfinite(dLdP[i])) throw Error(RVE_EINVAL, "non-finite loss weight");
    HIPCHECK(hipSetDevice(h->device));
    RVE& R = *h->rves[rve];
    if (R.increments < 1) throw Error(RVE_ESTATE, "no committed increment to reverse");
    Work& w = work(R, false);
    if (!w.plane) throw Error(RVE_EINVAL, "the reverse pass needs the plane kernels (grid planes do not fit in LDS)");
    if (R.freq != FREQ_ROTATED) throw Error(RVE_EINVAL, "the reverse pass needs the rotated-scheme frequencies");
    const int64_t nv = R.nvox;
    const size_t f9 = sizeof(double) * 9 * nv, f12 = sizeof(double) * 12 * nv;
    const int64_t nb = (nv + 63) / 64;
    if (!R.adj_a9.p) {
      R.adj_a9.alloc(f9);
      R.adj_b9.alloc(f9);
      R.adj_rgb.alloc(f12);
      R.adj_theta.alloc(sizeof(double) * 4 * nb);
    }
    hipStream_t st = R.stream;
    // 1. the converged state of the increment, re-evaluated from its start-of-increment state
    //    (the stored slip increments are the warm start): stress, slip increments, tangent
    HIPCHECK(hipMemcpyAsync(R.dg_saved.p, R.dg.p, f12, hipMemcpyDeviceToDevice, st));
    ConstArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nvox = nv;
    a.gid = R.d_gid.as<int32_t>();
    a.grainR = R.d_R.as<double>();
    a.grainC = R.d_C.as<double>();
    a.mat = R.d_mat.as<MatDev>();
    a.F = R.F.as<double>();
    a.Fp_n = R.Fp_prev.as<double>();
    a.rho_ssd = R.rho_ssd_prev.as<double>();
    a.rho_gnd = R.rho_gnd_prev.as<double>();
    a.dg = R.dg_saved.as<double>();
    a.P = R.P_work.as<double>();
    a.K = w.K.p;
    a.k_grouped = 1;
    a.k_inv_scale = 1.0;
    a.dt = R.dt_last;
    a.stats = R.blk.as<int32_t>();
    a.work = R.blk.as<int32_t>() + 4;
    launch_constitutive(a, KT_F64, st);
    check_launch("reverse pass: constitutive");
    int32_t st4[4];
    HIPCHECK(hipMemcpyAsync(st4, R.blk.p, sizeof(st4), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    if (st4[1] != 0) throw Error(RVE_ENOCONV, "local Newton did not converge at the committed state");
    w.k_ready = true;
    // 2. right-hand side of the adjoint equilibrium: g = dL/dF at fixed start state
    AdjointLocalArgs b;
    std::memset(&b, 0, sizeof(b));
    for (int i = 0; i < 9; ++i) b.wP[i] = dLdP[i] / (double)nv;
    b.Fp_bar = Fp_bar;
    b.rho_bar = rho_bar;
    b.g = R.adj_a9.as<double>();
    b.mode = 0;
    launch_constitutive_adjoint(a, b, st);
    check_launch("reverse pass: right-hand side");
    // 3. multiplier: G(K^T : lam) = G(g), lam in the range of G (r = -G(g), x = -lam)
    double keep[9];
    for (int c = 0; c < 9; ++c) keep[c] = mask[c] ? 0.0 : 1.0;
    void* x = w.xa.p;
    run_residual(*h, R, w, R.adj_a9.as<double>(), keep, nullptr, x);
    int done = 0;
    const int ncg = run_cg(*h, R, w, x, keep, done, true);
    if (cg_iters) *cg_iters = ncg;
    if (!(done == 1 || done == 5)) throw Error(RVE_ENOCONV, "adjoint conjugate gradients did not converge");
    launch_negate(static_cast<const double*>(x), R.adj_b9.as<double>(), 9 * nv, st);
    // 4. dL/d(start-of-increment state, parameters) at fixed F with P_bar = dL/dP - lam
    b.mode = 1;
    b.lam = R.adj_b9.as<double>();
    b.g = nullptr;
    b.Fp_bar_out = Fp_bar;
    b.rho_bar_out = rho_bar;
    b.rho_gnd_bar = R.adj_rgb.as<double>();
    b.theta_partial = R.adj_theta.as<double>();
    const int nblk = launch_constitutive_adjoint(a, b, st);
    check_launch("reverse pass: state and parameters");
    // 5. the start-of-increment GND densities came from the curl of Fp_{k-1} (eqs. 10-13):
    //    Fp_bar += curl^T (d rho_GND / d alpha)^T rho_gnd_bar at alpha = curl(Fp_{k-1})
    if (R.mat.hardening && R.mat.c_gnd != 0.0) {
      const GridPlan& g = w.plan.g;
      curl_plane64(g, w.spec.p, R.Fp_prev.as<double>(), true, 1.0 / R.h, R.adj_a9.as<double>(), st);
      launch_gnd_adjoint(nv, R.adj_a9.as<double>(), R.d_gid.as<int32_t>(), R.d_R.as<double>(), R.d_mat.as<MatDev>(),
                         R.adj_rgb.as<double>(), R.adj_b9.as<double>(), st);
      curl_plane64(g, w.spec.p, R.adj_b9.as<double>(), false, 1.0 / R.h, R.adj_a9.as<double>(), st);
      launch_roll_back(g.nx, g.ny, g.nz, R.adj_a9.as<double>(), Fp_bar, st, true);
      check_launch("reverse pass: GND chain");
    }
    // 6. parameter derivatives: block partials summed in a fixed order
    std::vector<double> part(4 * (size_t)nblk);
    HIPCHECK(hipMemcpyAsync(part.data(), R.adj_theta.p, sizeof(double) * part.size(), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    double th[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < nblk; ++i)
      for (int j = 0; j < 4; ++j) th[j] += part[4 * (size_t)i + j];
    theta_bar[1] += th[0];  // K
    theta_bar[2] += th[1];  // y_c
    theta_bar[3] += th[2];  // c_gnd
    theta_bar[0] += th[3];  // tau0 (tau_c held at tau0 without hardening)
    // 7. first increment: rho_SSD,0 = rho0 = (tau0 / (mu b))^2 / sum_b q^{ab} (uniform), so
    //    d rho0 / d tau0 = 2 rho0 / tau0 with tau0 = mu b sqrt(sum_b q^{ab} rho0)
    if (R.increments == 1 && R.mat.hardening) {
      double rs[12];
      field_average(*h, R, rho_bar, 12, rs);
      double sum = 0.0;
      for (int c = 0; c < 12; ++c) sum += rs[c] * (double)nv;
      double rowsum = 0.0;
      for (int c = 0; c < 12; ++c) rowsum += R.mat.q[c];
      const double tau0 = R.mat.mu * R.mat.burgers * std::sqrt(rowsum * R.rho0);
      theta_bar[0] += sum * 2.0 * R.rho0 / tau0;
    }
    return RVE_OK;
  });
}

// state: per RVE F, F_prev, Fp, Nye, P (9 each), rho_ssd, rho_gnd, dg (12 each), the
// start-of-increment Fp (9), rho_ssd, rho_gnd (12 each), followed by the host scalars.
int64_t rve_state_bytes(rve_handle h) {
  if (!h) return 0;
  int64_t b = 0;
  for (auto& r : h->rves) b += (int64_t)sizeof(double) * (9 * 6 + 12 * 5) * r->nvox + (int64_t)sizeof(double) * 48;
  return b;
}

int32_t rve_save_state(rve_handle h, void* buf) {
  return guarded([&]() -> int32_t {
    if (!h || !buf) throw Error(RVE_EINVAL, "null argument");
    HIPCHECK(hipSetDevice(h->device));
    char* o = (char*)buf;
    for (auto& rp : h->rves) {
      RVE& R = *rp;
      const DevBuf* bufs[11] = {&R.F,       &R.F_prev, &R.Fp,      &R.nye,          &R.P,           &R.rho_ssd,
                                &R.rho_gnd, &R.dg,     &R.Fp_prev, &R.rho_ssd_prev, &R.rho_gnd_prev};
      const int nc[11] = {9, 9, 9, 9, 9, 12, 12, 12, 9, 12, 12};
      for (int i = 0; i < 11; ++i) {
        const size_t n = sizeof(double) * nc[i] * R.nvox;
        HIPCHECK(hipMemcpyAsync(o, bufs[i]->p, n, hipMemcpyDeviceToHost, R.stream));
        o += n;
      }
      double sc[48] = {0};
      std::memcpy(sc, R.Favg, 72);
      std::memcpy(sc + 9, R.Favg_prev, 72);
      std::memcpy(sc + 18, R.Pavg, 72);
      std::memcpy(sc + 27, R.Fbar_prev, 72);
      sc[36] = R.have_prev ? 1.0 : 0.0;
      sc[37] = (double)R.increments;
      sc[38] = R.dt_last;
      std::memcpy(sc + 39, R.Pbar_prev, 72);
      std::memcpy(o, sc, sizeof(sc));
      o += sizeof(sc);
      HIPCHECK(hipStreamSynchronize(R.stream));
    }
    return RVE_OK;
  });
}

int32_t rve_load_state(rve_handle h, const void* buf) {
  return guarded([&]() -> int32_t {
    if (!h || !buf) throw Error(RVE_EINVAL, "null argument");
    HIPCHECK(hipSetDevice(h->device));
    const char* o = (const char*)buf;
    for (auto& rp : h->rves) {
      RVE& R = *rp;
      DevBuf* bufs[11] = {&R.F,       &R.F_prev, &R.Fp,      &R.nye,          &R.P,           &R.rho_ssd,
                          &R.rho_gnd, &R.dg,     &R.Fp_prev, &R.rho_ssd_prev, &R.rho_gnd_prev};
      const int nc[11] = {9, 9, 9, 9, 9, 12, 12, 12, 9, 12, 12};
      for (int i = 0; i < 11; ++i) {
        const size_t n = sizeof(double) * nc[i] * R.nvox;
        HIPCHECK(hipMemcpyAsync(bufs[i]->p, o, n, hipMemcpyHostToDevice, R.stream));
        o += n;
      }
      double sc[48];
      std::memcpy(sc, o, sizeof(sc));
      o += sizeof(sc);
      std::memcpy(R.Favg, sc, 72);
      std::memcpy(R.Favg_prev, sc + 9, 72);
      std::memcpy(R.Pavg, sc + 18, 72);
      std::memcpy(R.Fbar_prev, sc + 27, 72);
      R.have_prev = sc[36] != 0.0;
      R.increments = (int64_t)sc[37];
      R.dt_last = sc[38];
      std::memcpy(R.Pbar_prev, sc + 39, 72);
      // the tangents belong to whatever state was evaluated last, not to the loaded one
      R.w[0].k_ready = R.w[1].k_ready = false;
      HIPCHECK(hipStreamSynchronize(R.stream));
    }
    return RVE_OK;
  });
}

// ---- kernel-level entry points ------------------------------------------------------

int32_t rve_constitutive_batch(const rve_material* mat, int32_t n_grains, const double* grain_quat, int64_t nvox,
                               const int32_t* gid, const double* F, const double* Fp_n, const double* rho_ssd_n,
                               const double* rho_gnd_n, double dt, double* dg, double* P, double* K, int32_t* iters,
                               void* stream) {
  return guarded([&]() -> int32_t {
    if (!mat || n_grains < 1 || !grain_quat || nvox < 1 || !gid || !F || !Fp_n || !rho_ssd_n || !rho_gnd_n || !dg ||
        !P)
      throw Error(RVE_EINVAL, "null argument");
    if (!(std::isfinite(dt) && dt > 0)) throw Error(RVE_EINVAL, "dt must be > 0");
    hipStream_t st = (hipStream_t)stream;
    MatDev md = make_material(*mat);
    std::vector<double> Rg(9 * (size_t)n_grains);
    for (int g = 0; g < n_grains; ++g) quat_to_R(grain_quat + 4 * g, &Rg[9 * g]);
    DevBuf dmat, dR, Kc, cnt;
    cnt.alloc(sizeof(int32_t) * (4 + nvox));
    upload(dmat, &md, sizeof(md));
    upload(dR, Rg.data(), sizeof(double) * Rg.size());
    if (K) Kc.alloc(sizeof(double) * 81 * nvox);
    ConstArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nvox = nvox;
    a.gid = gid;
    a.grainR = dR.as<double>();
    a.mat = dmat.as<MatDev>();
    a.F = F;
    a.Fp_n = Fp_n;
    a.rho_ssd = rho_ssd_n;
    a.rho_gnd = rho_gnd_n;
    a.dg = dg;
    a.P = P;
    a.K = K ? Kc.p : nullptr;
    a.dt = dt;
    a.iters = iters;
    a.stats = cnt.as<int32_t>();
    a.work = cnt.as<int32_t>() + 4;
    launch_constitutive(a, KT_F64, st);
    check_launch("constitutive");
    if (K) {
      launch_rotate_tangent(nvox, gid, dR.as<double>(), Kc.as<double>(), K, st);
      check_launch("rotate tangent");
    }
    HIPCHECK(hipStreamSynchronize(st));
    return RVE_OK;
  });
}

static void stress_sensitivity(const rve_material* mat, int32_t n_grains, const double* grain_quat, int64_t nvox,
                               const int32_t* gid, const double* F, const double* Fp_n, const double* rho_ssd_n,
                               const double* rho_gnd_n, double dt, const double* dg, const double* w, double* out,
                               hipStream_t st) {
  if (!mat || n_grains < 1 || !grain_quat || nvox < 1 || !gid || !F || !Fp_n || !rho_ssd_n || !rho_gnd_n || !dg ||
      !out)
    throw Error(RVE_EINVAL, "null argument");
  if (!(std::isfinite(dt) && dt > 0)) throw Error(RVE_EINVAL, "dt must be > 0");
  MatDev md = make_material(*mat);
  std::vector<double> Rg(9 * (size_t)n_grains);
  for (int g = 0; g < n_grains; ++g) quat_to_R(grain_quat + 4 * g, &Rg[9 * g]);
  DevBuf dmat, dR;
  upload(dmat, &md, sizeof(md));
  upload(dR, Rg.data(), sizeof(double) * Rg.size());
  ConstArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nvox = nvox;
  a.gid = gid;
  a.grainR = dR.as<double>();
  a.mat = dmat.as<MatDev>();
  a.F = F;
  a.Fp_n = Fp_n;
  a.rho_ssd = rho_ssd_n;
  a.rho_gnd = rho_gnd_n;
  a.dg = const_cast<double*>(dg);   // read only
  a.dt = dt;
  launch_stress_sensitivity(a, out, w, st);
  check_launch("stress sensitivity");
  HIPCHECK(hipStreamSynchronize(st));
}

int32_t rve_stress_sensitivity(const rve_material* mat, int32_t n_grains, const double* grain_quat, int64_t nvox,
                               const int32_t* gid, const double* F, const double* Fp_n, const double* rho_ssd_n,
                               const double* rho_gnd_n, double dt, const double* dg, double* dPdtc,
                               void* stream) {
  return guarded([&]() -> int32_t {
    stress_sensitivity(mat, n_grains, grain_quat, nvox, gid, F, Fp_n, rho_ssd_n, rho_gnd_n, dt, dg, nullptr, dPdtc,
                       (hipStream_t)stream);
    return RVE_OK;
  });
}

int32_t rve_stress_sensitivity_vjp(const rve_material* mat, int32_t n_grains, const double* grain_quat,
                                   int64_t nvox, const int32_t* gid, const double* F, const double* Fp_n,
                                   const double* rho_ssd_n, const double* rho_gnd_n, double dt, const double* dg,
                                   const double* w, double* tau_c_bar, void* stream) {
  return guarded([&]() -> int32_t {
    if (!w) throw Error(RVE_EINVAL, "null argument");
    stress_sensitivity(mat, n_grains, grain_quat, nvox, gid, F, Fp_n, rho_ssd_n, rho_gnd_n, dt, dg, w, tau_c_bar,
                       (hipStream_t)stream);
    return RVE_OK;
  });
}

int32_t rve_density_sensitivity(const rve_material* mat, int64_t nvox, const double* rho_ssd_n,
                                const double* rho_gnd_n, const double* dg, double* out, void* stream) {
  return guarded([&]() -> int32_t {
    if (!mat || nvox < 1 || !rho_ssd_n || !rho_gnd_n || !dg || !out) throw Error(RVE_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    MatDev md = make_material(*mat);
    DevBuf dmat;
    upload(dmat, &md, sizeof(md));
    launch_density_sensitivity(nvox, dmat.as<MatDev>(), rho_ssd_n, rho_gnd_n, dg, out, st);
    check_launch("density sensitivity");
    HIPCHECK(hipStreamSynchronize(st));
    return RVE_OK;
  });
}

int32_t rve_project(const int32_t n[3], int32_t precision, const double* A, const uint8_t* mask,
                    const double* dc_target, double* out, void* stream) {
  return guarded([&]() -> int32_t {
    if (!n || !A || !mask || !out) throw Error(RVE_EINVAL, "null argument");
    prepare_device();
    const bool fp32 = precision == RVE_MIXED;
    hipStream_t st = (hipStream_t)stream;
    Plan P;
    build_plan(P, n, fp32);
    const GridPlan& g = P.g;
    DevBuf spec;
    spec.alloc(tsize(fp32) * 2 * 9 * g.nspec);
    const bool plane = plane_enabled() && plane_fits(g, fp32);
    double keep[9];
    for (int c = 0; c < 9; ++c) keep[c] = mask[c] ? 0.0 : 1.0;
    project_field(g, fp32, plane, spec.p, A, keep, dc_target, out, st);
    check_launch("project");
    HIPCHECK(hipStreamSynchronize(st));
    return RVE_OK;
  });
}

int32_t rve_spectral_curl(const int32_t n[3], int32_t precision, double h, const double* Fp, double* nye,
                          const int32_t* gid, int32_t n_grains, const double* grain_quat, double burgers,
                          double* rho_gnd, void* stream) {
  return guarded([&]() -> int32_t {
    if (!n || !Fp || !nye) throw Error(RVE_EINVAL, "null argument");
    if (!(std::isfinite(h) && h > 0)) throw Error(RVE_EINVAL, "h must be > 0");
    prepare_device();
    const bool fp32 = precision == RVE_MIXED;
    hipStream_t st = (hipStream_t)stream;
    Plan P;
    build_plan(P, n, fp32);
    const GridPlan& g = P.g;
    DevBuf spec, dmat, dR;
    spec.alloc(tsize(fp32) * 2 * 9 * g.nspec);
    const bool gnd = rho_gnd && gid && grain_quat && n_grains > 0;
    if (gnd) {
      if (!(burgers > 0)) throw Error(RVE_EINVAL, "burgers must be > 0");
      MatDev md;
      std::memset(&md, 0, sizeof(md));
      md.burgers = burgers;
      segment_pinv(md.Aplus, md.screw_of);
      std::vector<double> Rg(9 * (size_t)n_grains);
      for (int gi = 0; gi < n_grains; ++gi) quat_to_R(grain_quat + 4 * gi, &Rg[9 * gi]);
      upload(dmat, &md, sizeof(md));
      upload(dR, Rg.data(), sizeof(double) * Rg.size());
    }
    const bool plane = plane_enabled() && plane_fits(g, fp32);
    if (plane) {
      PlaneArgs pa{PF_FPI, Fp, spec.p};
      launch_plane_fwd(g, fp32, pa, nullptr, st);
    } else {
      XFwdArgs xf;
      std::memset(&xf, 0, sizeof(xf));
      xf.mode = XF_FP_MINUS_I;
      xf.in64 = Fp;
      xf.spec = spec.p;
      launch_xfwd(g, fp32, xf, st);
      launch_yfft(g, fp32, spec.p, -1, nullptr, st);
    }
    MidArgs m;
    std::memset(&m, 0, sizeof(m));
    m.op = MID_CURL;
    m.spec = spec.p;
    m.inv_n = 1.0 / (double)g.nvox;
    m.inv_h = 1.0 / h;
    launch_mid(g, fp32, m, st);
    if (plane) {
      PlaneInvArgs pi;
      std::memset(&pi, 0, sizeof(pi));
      pi.mode = PI_OUT64;
      pi.spec = spec.p;
      pi.out64 = nye;
      launch_plane_inv(g, fp32, pi, st);
      if (gnd) launch_gnd(g.nvox, nye, gid, dR.as<double>(), dmat.as<MatDev>(), rho_gnd, st);
      check_launch("curl");
      HIPCHECK(hipStreamSynchronize(st));
      return RVE_OK;
    }
    launch_yfft(g, fp32, spec.p, +1, nullptr, st);
    XInvArgs xi;
    std::memset(&xi, 0, sizeof(xi));
    xi.mode = XI_NYE;
    xi.spec = spec.p;
    xi.out64 = nye;
    if (gnd) {
      xi.rho_gnd = rho_gnd;
      xi.gid = gid;
      xi.grainR = dR.as<double>();
      xi.mat = dmat.as<MatDev>();
    }
    launch_xinv(g, fp32, xi, st);
    check_launch("curl");
    HIPCHECK(hipStreamSynchronize(st));
    return RVE_OK;
  });
}

int32_t rve_gnd_adjoint(const int32_t n[3], int32_t precision, double h, const double* nye, const int32_t* gid,
                        int32_t n_grains, const double* grain_quat, double burgers, const double* rho_bar,
                        double* nye_bar, double* Fp_bar, void* stream) {
  return guarded([&]() -> int32_t {
    if (!n || !nye || !gid || !grain_quat || !rho_bar || !Fp_bar) throw Error(RVE_EINVAL, "null argument");
    if (n_grains < 1) throw Error(RVE_EINVAL, "n_grains must be >= 1");
    if (!(std::isfinite(h) && h > 0)) throw Error(RVE_EINVAL, "h must be > 0");
    if (!(std::isfinite(burgers) && burgers > 0)) throw Error(RVE_EINVAL, "burgers must be > 0");
    prepare_device();
    const bool fp32 = precision == RVE_MIXED;
    hipStream_t st = (hipStream_t)stream;
    Plan P;
    build_plan(P, n, fp32);
    const GridPlan& g = P.g;
    const size_t f9 = sizeof(double) * 9 * (size_t)g.nvox;
    DevBuf spec, dmat, dR, abar, curl;
    spec.alloc(tsize(fp32) * 2 * 9 * g.nspec);
    curl.alloc(f9);
    double* ab = nye_bar;
    if (!ab) {
      abar.alloc(f9);
      ab = abar.as<double>();
    }
    MatDev md;
    std::memset(&md, 0, sizeof(md));
    md.burgers = burgers;
    segment_pinv(md.Aplus, md.screw_of);
    std::vector<double> Rg(9 * (size_t)n_grains);
    for (int gi = 0; gi < n_grains; ++gi) quat_to_R(grain_quat + 4 * gi, &Rg[9 * gi]);
    upload(dmat, &md, sizeof(md));
    upload(dR, Rg.data(), sizeof(double) * Rg.size());
    launch_gnd_adjoint(g.nvox, nye, gid, dR.as<double>(), dmat.as<MatDev>(), rho_bar, ab, st);
    // transposed curl: the forward spectral curl of alpha_bar, then one voxel back per axis
    const bool plane = plane_enabled() && plane_fits(g, fp32);
    if (plane) {
      PlaneArgs pa{PF_F64, ab, spec.p};
      launch_plane_fwd(g, fp32, pa, nullptr, st);
    } else {
      XFwdArgs xf;
      std::memset(&xf, 0, sizeof(xf));
      xf.mode = XF_FIELD64;
      xf.in64 = ab;
      xf.spec = spec.p;
      launch_xfwd(g, fp32, xf, st);
      launch_yfft(g, fp32, spec.p, -1, nullptr, st);
    }
    MidArgs m;
    std::memset(&m, 0, sizeof(m));
    m.op = MID_CURL;
    m.spec = spec.p;
    m.inv_n = 1.0 / (double)g.nvox;
    m.inv_h = 1.0 / h;
    launch_mid(g, fp32, m, st);
    if (plane) {
      PlaneInvArgs pi;
      std::memset(&pi, 0, sizeof(pi));
      pi.mode = PI_OUT64;
      pi.spec = spec.p;
      pi.out64 = curl.as<double>();
      launch_plane_inv(g, fp32, pi, st);
    } else {
      launch_yfft(g, fp32, spec.p, +1, nullptr, st);
      XInvArgs xi;
      std::memset(&xi, 0, sizeof(xi));
      xi.mode = XI_OUT64;
      xi.spec = spec.p;
      xi.out64 = curl.as<double>();
      launch_xinv(g, fp32, xi, st);
    }
    launch_roll_back(g.nx, g.ny, g.nz, curl.as<double>(), Fp_bar, st);
    check_launch("gnd adjoint");
    HIPCHECK(hipStreamSynchronize(st));
    return RVE_OK;
  });
}

int32_t rve_project_noalloc(const int32_t n[3], int32_t precision, const double* A, const uint8_t* mask,
                            const double* dc_target, double* out, void* stream) {
  return guarded([&]() -> int32_t {
    if (!n || !A || !mask || !out) throw Error(RVE_EINVAL, "null argument");
    if (precision != RVE_FP64 && precision != RVE_MIXED) throw Error(RVE_EINVAL, "unknown precision");
    const int nn[3] = {n[0], n[1], n[2]};
    const bool fp32 = precision == RVE_MIXED;
    GridPlan g;
    void* spec = nullptr;
    noalloc_plan(g, nn, fp32, nullptr, &spec);  // shape and size checks, host only
    prepare_device();
    unsigned char* base = static_cast<unsigned char*>(noalloc_base());
    noalloc_plan(g, nn, fp32, base, &spec);
    hipStream_t st = (hipStream_t)stream;
    const int* dims[3] = {&g.nx, &g.ny, &g.nz};
    const void* tw[3] = {g.twx, g.twy, g.twz};
    const void* E[3] = {g.Ex, g.Ey, g.Ez};
    for (int d = 0; d < 3; ++d) {
      const int m = *dims[d];
      if (fp32)
        hipLaunchKernelGGL(k_root_tables<float>, dim3((m + 255) / 256), dim3(256), 0, st, m,
                           (float*)const_cast<void*>(tw[d]), (double*)const_cast<void*>(E[d]));
      else
        hipLaunchKernelGGL(k_root_tables<double>, dim3((m + 255) / 256), dim3(256), 0, st, m,
                           (double*)const_cast<void*>(tw[d]), (double*)const_cast<void*>(E[d]));
    }
    check_launch("root tables");
    double keep[9];
    for (int c = 0; c < 9; ++c) keep[c] = mask[c] ? 0.0 : 1.0;
    project_field(g, fp32, plane_enabled() && plane_fits(g, fp32), spec, A, keep, dc_target, out, st);
    check_launch("project (no allocation)");
    return RVE_OK;
  });
}

}  // extern "C"
