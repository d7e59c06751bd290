// C ABI of the library: plan / problem objects, workspace carving, and the
// orchestration of set-up, factorisation and the GMRES solve.  Every O(N)
// step runs in the HIP kernels of the other translation units; this file only
// sequences launches on the problem's stream and reads back per-right-hand-
// side scalars for the GMRES control decisions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "krylov.h"
#include <map>
#include <mutex>
#include <tuple>

#include "lsp_common.h"
#include "plan.h"
#include "static_scratch.h"

using namespace lsp;

// Device copy of a plan's constant arrays (front descriptors, index lists,
// extend-add maps, class geometry, FFT twiddles), one per device the plan is
// used on: uploaded once, at the first lsp_setup on that device.
struct PlanDev {
  void* block = nullptr;
  FrontDev* fronts = nullptr;
  int* idx = nullptr;
  unsigned* gpos = nullptr;
  int* cpos = nullptr;
  ClassGeom* geo = nullptr;
  double2* tw64 = nullptr;
  float2* tw32 = nullptr;
  int* ptab = nullptr;        // general domains: Plan::ptab, bpts, bslots
  int* bpts = nullptr;
  unsigned* bslots = nullptr;
};

struct lsp_plan {
  Plan p;
  std::vector<ClassGeom> geo;
  int nclass = 0;
  long long maxF = 0;
  int gram_blocks = 1;
  mutable std::mutex dev_mu;
  mutable std::map<int, PlanDev> dev;
  ~lsp_plan() {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return;
    for (auto& kv : dev) {
      if (hipSetDevice(kv.first) == hipSuccess) (void)hipFree(kv.second.block);
    }
    (void)hipSetDevice(cur);
  }
};

namespace {

thread_local std::string g_last_error;

lsp_status fail(lsp_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

template <typename F>
lsp_status guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return fail(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail(LSP_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(LSP_ERR_HIP, e.what());
  }
}

// Bump allocator over a caller-provided device workspace.  With base == null
// it only measures.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct ProblemPtrs {
  double2* ktab;
  double2* spec64;  // spectrum rows in the K-matvec's split order
  float2* spec32;
  double2* tw64;
  float2* tw32;
  double* w2m;
  double2* Mval;
  ClassGeom* geo;
  double2* alpha_pad;
  double2* C_pad;
  double* sigma_pad;
  double2* G;
  double2* U1;
  double2* partial;
  double2* E;
  void* F;
  void* Dinv;
  FrontDev* fronts;
  int* idx;
  unsigned* gpos;
  int* cpos;
  int* perm;
  double* pivstat;
  void* Gop;  // formed dense sweep operators
  // general domains: the sketch T = (K w^2 m) R (r rows of N), the boundary
  // points' stencils and singular values ([nbnd][27]), the output mask, and
  // the plan's point tables
  double2* T;
  double2* Tw;      // the sketch products' FFT work array, kSketchBatch columns
  double2* balpha;
  double* bsigma;
  double* dmask;
  int* ptab;
  int* bpts;
  unsigned* bslots;
};

constexpr int kSketchBatch = 8;  // sketch columns per batched K product

size_t layout_problem(const lsp_plan* pl, int precision, void* base, ProblemPtrs* out) {
  const Plan& P = pl->p;
  Carver cv(base);
  ProblemPtrs q{};
  long long n1d = 1, hd = P.L, Ld = 1;
  for (int a = 0; a < P.d; ++a) { n1d *= P.n + 1; Ld *= P.L; }
  for (int a = 1; a < P.d; ++a) hd *= P.n + 1;
  const int S = kMaxStencil;
  q.ktab = cv.take<double2>(n1d);
  q.spec64 = cv.take<double2>(hd);
  q.spec32 = cv.take<float2>(hd);
  q.w2m = cv.take<double>(P.N);
  q.Mval = cv.take<double2>((size_t)P.N * (P.d == 2 ? 9 : 27));
  q.alpha_pad = cv.take<double2>((size_t)pl->nclass * S);
  q.C_pad = cv.take<double2>((size_t)pl->nclass * S);
  q.sigma_pad = cv.take<double>((size_t)pl->nclass * S);
  q.G = cv.take<double2>((size_t)pl->nclass * S * S);
  q.U1 = cv.take<double2>((size_t)pl->nclass * S * S);
  q.partial = cv.take<double2>((size_t)pl->gram_blocks * pl->nclass * S * S);
  q.E = cv.take<double2>(Ld);
  size_t esz = precision == LSP_MIXED ? sizeof(float2) : sizeof(double2);
  q.F = cv.take<char>((size_t)P.front_elems * esz);
  q.Dinv = cv.take<char>((size_t)P.dinv_elems * esz);
  q.perm = cv.take<int>(P.sum_p);
  q.pivstat = cv.take<double>((size_t)P.panel_blocks);
  q.Gop = cv.take<char>((size_t)P.dense_elems * esz);
  if (P.general) {
    q.T = cv.take<double2>((size_t)P.sketch_r * P.N);
    q.Tw = cv.take<double2>((size_t)std::min(P.sketch_r, kSketchBatch) * Ld);
    q.balpha = cv.take<double2>(std::max<size_t>(1, P.bpts.size()) * S);
    q.bsigma = cv.take<double>(std::max<size_t>(1, P.bpts.size()) * S);
    q.dmask = cv.take<double>(P.N);
  }
  if (out) *out = q;
  return cv.off + 256;
}

// The plan's device copy on `device` (current), created on first use.
const PlanDev& plan_device(const lsp_plan* pl, int device) {
  std::lock_guard<std::mutex> lock(pl->dev_mu);
  auto it = pl->dev.find(device);
  if (it != pl->dev.end()) return it->second;
  const Plan& P = pl->p;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t bf = up(P.fronts.size() * sizeof(FrontDev)), bi = up(P.idx.size() * sizeof(int)),
               bp = up(P.gpos.size() * sizeof(unsigned)), bc = up(P.cpos.size() * sizeof(int)),
               bg = up(pl->geo.size() * sizeof(ClassGeom)), bt = up(P.L * sizeof(double2)),
               bt32 = up(P.L * sizeof(float2)), bpt = up(P.ptab.size() * sizeof(int)),
               bbp = up(P.bpts.size() * sizeof(int)), bbs = up(P.bslots.size() * sizeof(unsigned));
  PlanDev d;
  if (hipMalloc(&d.block, bf + bi + bp + bc + bg + bt + bt32 + bpt + bbp + bbs) != hipSuccess) {
    (void)hipGetLastError();
    throw Error(LSP_ERR_OOM, "device allocation of the plan arrays failed");
  }
  char* b = (char*)d.block;
  d.fronts = (FrontDev*)b; b += bf;
  d.idx = (int*)b; b += bi;
  d.gpos = (unsigned*)b; b += bp;
  d.cpos = (int*)b; b += bc;
  d.geo = (ClassGeom*)b; b += bg;
  d.tw64 = (double2*)b; b += bt;
  d.tw32 = (float2*)b; b += bt32;
  if (P.general) {
    d.ptab = (int*)b; b += bpt;
    d.bpts = (int*)b; b += bbp;
    d.bslots = (unsigned*)b;
  }
  // twiddles exp(-2 pi i k / L) from long double
  std::vector<double2> tw64(P.L);
  std::vector<float2> tw32(P.L);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < P.L; ++k) {
    long double a = 2.0L * pi * (long double)k / (long double)P.L;
    tw64[k] = make_double2((double)cosl(a), (double)-sinl(a));
    tw32[k] = make_float2((float)cosl(a), (float)-sinl(a));
  }
  try {
    LSP_HIP(hipMemcpy(d.fronts, P.fronts.data(), P.fronts.size() * sizeof(FrontDev), hipMemcpyHostToDevice));
    LSP_HIP(hipMemcpy(d.idx, P.idx.data(), P.idx.size() * sizeof(int), hipMemcpyHostToDevice));
    LSP_HIP(hipMemcpy(d.gpos, P.gpos.data(), P.gpos.size() * sizeof(unsigned), hipMemcpyHostToDevice));
    LSP_HIP(hipMemcpy(d.cpos, P.cpos.data(), P.cpos.size() * sizeof(int), hipMemcpyHostToDevice));
    LSP_HIP(hipMemcpy(d.geo, pl->geo.data(), pl->geo.size() * sizeof(ClassGeom), hipMemcpyHostToDevice));
    LSP_HIP(hipMemcpy(d.tw64, tw64.data(), P.L * sizeof(double2), hipMemcpyHostToDevice));
    LSP_HIP(hipMemcpy(d.tw32, tw32.data(), P.L * sizeof(float2), hipMemcpyHostToDevice));
    if (P.general) {
      LSP_HIP(hipMemcpy(d.ptab, P.ptab.data(), P.ptab.size() * sizeof(int), hipMemcpyHostToDevice));
      if (!P.bpts.empty()) {
        LSP_HIP(hipMemcpy(d.bpts, P.bpts.data(), P.bpts.size() * sizeof(int), hipMemcpyHostToDevice));
        LSP_HIP(hipMemcpy(d.bslots, P.bslots.data(), P.bslots.size() * sizeof(unsigned), hipMemcpyHostToDevice));
      }
    }
    // a copy from pageable memory may return before its DMA has landed, and
    // the problems' streams do not wait for the null stream
    LSP_HIP(hipDeviceSynchronize());
  } catch (...) {
    (void)hipFree(d.block);
    throw;
  }
  return pl->dev.emplace(device, d).first->second;
}

struct SolvePtrs {
  void* W;        // FFT work [nrhs][L^d] complex128-sized
  void* vbuf;     // front vectors [nrhs][sum(p+q)]
  void* zq;       // Q-apply output [nrhs][N]
  void* xs;       // M^{-1} output [nrhs][N]
  void* ybuf;     // blocked sweeps: super-block outputs [nrhs][bsweep_ystride]
  void* pbuf;     // blocked sweeps: boundary partial sums [chunks][nrhs][bsweep_ystride]
  void* xpm;      // matrix-core levels: the solution point-major, [ceil(nrhs/16)][N][16]
  double2* V;     // [restart+1][nrhs][N]
  double2* Z;     // [restart][nrhs][N]
  double2* w;     // [nrhs][N]
  double2* g;
  double2* r;
  double2* t;
  double2* H;     // [nrhs][(restart+1) restart]
  double2* cs;
  double2* sn;
  double2* gam;
  double2* h;     // [nrhs][kMaxVec]
  double2* y;
  double2* partial;
  double2* partial2;
  double* scal;   // [nrhs][kScal]
  int* active;
  int* ksz;
  int* iters;
  int* done;
};

size_t layout_solve(const Plan& P, int nrhs, int restart, bool krylov, void* base, SolvePtrs* out) {
  Carver cv(base);
  SolvePtrs s{};
  long long Ld = 1;
  for (int a = 0; a < P.d; ++a) Ld *= P.L;
  const size_t N = P.N;
  s.W = cv.take<double2>((size_t)nrhs * Ld);
  s.vbuf = cv.take<double2>((size_t)nrhs * P.sum_pq);
  s.zq = cv.take<double2>((size_t)nrhs * N);
  s.xs = cv.take<double2>((size_t)nrhs * N);
  s.ybuf = cv.take<double2>((size_t)nrhs * P.bsweep_ystride);
  s.pbuf = cv.take<double2>((size_t)P.bsweep_chunks * nrhs * P.bsweep_ystride);
  s.xpm = cv.take<double2>(P.mchain_levels ? (size_t)((nrhs + 15) / 16) * 16 * N : 1);
  if (krylov) {
    s.V = cv.take<double2>((size_t)(restart + 1) * nrhs * N);
    s.Z = cv.take<double2>((size_t)restart * nrhs * N);
    s.w = cv.take<double2>((size_t)nrhs * N);
    s.g = cv.take<double2>((size_t)nrhs * N);
    s.r = cv.take<double2>((size_t)nrhs * N);
    s.t = cv.take<double2>((size_t)nrhs * N);
    s.H = cv.take<double2>((size_t)nrhs * (restart + 1) * restart);
    s.cs = cv.take<double2>((size_t)nrhs * restart);
    s.sn = cv.take<double2>((size_t)nrhs * restart);
    s.gam = cv.take<double2>((size_t)nrhs * (restart + 1));
    s.h = cv.take<double2>((size_t)nrhs * kMaxVec);
    s.y = cv.take<double2>((size_t)nrhs * kMaxVec);
    s.partial = cv.take<double2>((size_t)nrhs * dot_blocks((long long)N) * kMaxVec);
    s.partial2 = cv.take<double2>((size_t)nrhs * dot_blocks((long long)N) * kMaxVec);
    s.scal = cv.take<double>((size_t)nrhs * kScal);
    s.active = cv.take<int>(nrhs);
    s.ksz = cv.take<int>(nrhs);
    s.iters = cv.take<int>(nrhs);
    s.done = cv.take<int>(nrhs);
  }
  if (out) *out = s;
  return cv.off + 256;
}

}  // namespace

struct lsp_problem {
  const lsp_plan* plan = nullptr;
  int precision = LSP_FP64;
  double omega = 0.0;
  hipStream_t st = nullptr;
  int device = 0;
  ProblemPtrs d{};
  FftPlanDev<double> fp64{};
  FftPlanDev<float> fp32{};
  bool factored = false;
  double min_pivot_ratio = 0.0;
  // control block in pinned, coherent host memory (HostCtl, then iters,
  // est, beta, gnorm for host_cap right-hand sides), taken from a process-
  // wide pool so that creating a problem does not pin memory each time
  void* ctl_host = nullptr;
  void* ctl_dev = nullptr;
  int host_cap = 0;
  unsigned ctl_tag = 0;
  // formation stream (shared by the problems of a device) and this
  // problem's events for the dense levels' operator formation, taken at the
  // first factorisation that forms any; form_pending: the next sweeps must
  // wait for fs.done
  FormStream fs{};
  bool form_pending = false;
  // phase events (timing enabled) on the problem's stream: set-up, the last
  // factorisation and the last solve, each a start / end pair
  enum { EV_SETUP0, EV_SETUP1, EV_FACTOR0, EV_FACTOR1, EV_SOLVE0, EV_SOLVE1, EV_COUNT };
  hipEvent_t ev[EV_COUNT] = {};

  ~lsp_problem() {
    if (ev[0]) {
      (void)hipEventSynchronize(ev[EV_SETUP1]);
      std::lock_guard<std::mutex> g(event_pool_mu());
      for (hipEvent_t e : ev) event_pool().emplace_back(device, e);
    }
    if (ctl_host) ctl_pool().put({ctl_host, ctl_dev, host_cap});
    if (fs.aux) {
      // the caller may release the workspace next: the formation must be over
      (void)hipEventSynchronize(fs.done);
      form_pool().put(device, st, fs);
    }
  }

  // One formation stream per (device, problem stream), shared by the
  // problems that run on that stream (creating a stream costs milliseconds),
  // so that problems on different streams (serving slots) never wait for each
  // other's formation; and pooled event pairs.  All live until the process
  // ends.
  struct FormKey {
    int dev;
    hipStream_t user;
  };
  struct FormPool {
    std::mutex mu;
    std::vector<std::pair<FormKey, hipStream_t>> streams;
    std::vector<std::pair<FormKey, FormStream>> free;
    FormStream get(int dev, hipStream_t user) {
      std::lock_guard<std::mutex> g(mu);
      for (size_t i = 0; i < free.size(); ++i)
        if (free[i].first.dev == dev && free[i].first.user == user) {
          FormStream f = free[i].second;
          free.erase(free.begin() + i);
          return f;
        }
      FormStream f{};
      for (const auto& e : streams)
        if (e.first.dev == dev && e.first.user == user) f.aux = e.second;
      if (!f.aux) {
        LSP_HIP(hipStreamCreateWithFlags(&f.aux, hipStreamNonBlocking));
        streams.push_back({FormKey{dev, user}, f.aux});
      }
      LSP_HIP(hipEventCreateWithFlags(&f.level, hipEventDisableTiming));
      if (hipEventCreateWithFlags(&f.done, hipEventDisableTiming) != hipSuccess) {
        (void)hipEventDestroy(f.level);
        throw Error(LSP_ERR_HIP, "event creation for the formation stream failed");
      }
      LSP_HIP(hipEventRecord(f.done, f.aux));  // so that a first wait on it returns once the stream's work so far is done
      return f;
    }
    void put(int dev, hipStream_t user, const FormStream& f) {
      std::lock_guard<std::mutex> g(mu);
      free.push_back({FormKey{dev, user}, f});
    }
  };
  static FormPool& form_pool() {
    static FormPool* pool = new FormPool();
    return *pool;
  }
  // Timing events for the phases, pooled per device for the process's life.
  static std::mutex& event_pool_mu() {
    static std::mutex* m = new std::mutex();
    return *m;
  }
  static std::vector<std::pair<int, hipEvent_t>>& event_pool() {
    static auto* v = new std::vector<std::pair<int, hipEvent_t>>();
    return *v;
  }
  void take_events() {
    std::lock_guard<std::mutex> g(event_pool_mu());
    auto& pool = event_pool();
    for (int i = 0; i < EV_COUNT; ++i) {
      ev[i] = nullptr;
      for (size_t k = 0; k < pool.size(); ++k)
        if (pool[k].first == device) {
          ev[i] = pool[k].second;
          pool.erase(pool.begin() + k);
          break;
        }
      if (!ev[i]) LSP_HIP(hipEventCreate(&ev[i]));
    }
  }
  // milliseconds between two recorded events of this problem (0 if either
  // was never recorded)
  double phase_ms(int a, int b, bool recorded) const {
    float ms = 0.0f;
    if (!recorded || hipEventElapsedTime(&ms, ev[a], ev[b]) != hipSuccess) {
      (void)hipGetLastError();
      return 0.0;
    }
    return ms;
  }
  bool factor_timed = false;

  // the event the next sweeps wait for, once after each factorisation
  hipEvent_t take_form_wait() {
    if (!form_pending) return nullptr;
    form_pending = false;
    return fs.done;
  }

  static size_t ctl_bytes(int cap) { return sizeof(HostCtl) + 8 * (size_t)cap + 3 * sizeof(double) * (size_t)cap; }

  struct CtlBlock {
    void* host;
    void* dev;
    int cap;
  };
  // Blocks are returned only by destroyed problems, whose every report has
  // been waited for, so no device write to a pooled block is in flight.  The
  // pool lives until the process ends.
  struct CtlPool {
    std::mutex mu;
    std::vector<CtlBlock> free;
    CtlBlock get(int cap) {
      {
        std::lock_guard<std::mutex> g(mu);
        int best = -1;
        for (int i = 0; i < (int)free.size(); ++i)
          if (free[i].cap >= cap && (best < 0 || free[i].cap < free[best].cap)) best = i;
        if (best >= 0) {
          CtlBlock b = free[best];
          free.erase(free.begin() + best);
          return b;
        }
      }
      CtlBlock b{nullptr, nullptr, std::max(cap, 8)};
      LSP_HIP(hipHostMalloc(&b.host, ctl_bytes(b.cap),
                            hipHostMallocMapped | hipHostMallocCoherent | hipHostMallocPortable));
      const hipError_t e = hipHostGetDevicePointer(&b.dev, b.host, 0);
      if (e != hipSuccess) {
        (void)hipHostFree(b.host);
        LSP_HIP(e);
      }
      return b;
    }
    void put(const CtlBlock& b) {
      std::lock_guard<std::mutex> g(mu);
      free.push_back(b);
    }
  };
  static CtlPool& ctl_pool() {
    static CtlPool* pool = new CtlPool();
    return *pool;
  }

  static CtlView ctl_view(void* base, int cap) {
    char* b = static_cast<char*>(base);
    CtlView v;
    v.hdr = reinterpret_cast<HostCtl*>(b);
    v.iters = reinterpret_cast<int*>(b + sizeof(HostCtl));
    double* dv = reinterpret_cast<double*>(b + sizeof(HostCtl) + 8 * (size_t)cap);
    v.est = dv;
    v.beta = dv + cap;
    v.gnorm = dv + 2 * (size_t)cap;
    return v;
  }

  void ensure_host(int nrhs) {
    if (nrhs <= host_cap) return;
    const CtlBlock b = ctl_pool().get(nrhs);
    if (ctl_host) ctl_pool().put({ctl_host, ctl_dev, host_cap});
    ctl_host = b.host;
    ctl_dev = b.dev;
    host_cap = b.cap;
    std::memset(ctl_host, 0, ctl_bytes(host_cap));
    ctl_tag = 0;
  }

  // Waits until the device has reported `tag` (the stream's work up to the
  // reporting kernel is then done) and returns the number of right-hand
  // sides still iterating.  Polls the pinned block; every few thousand polls
  // it asks the stream for errors, and a stream that has finished without
  // the tag is an error.
  int wait_ctl(unsigned tag) {
    HostCtl* h = ctl_view(ctl_host, host_cap).hdr;
    long polls = 0, idle_polls = -1;
    while (__atomic_load_n(&h->tag, __ATOMIC_ACQUIRE) != tag) {
      if (idle_polls >= 0) {
        if (++idle_polls > (1L << 24)) throw Error(LSP_ERR_HIP, "solver control report did not arrive");
      } else if ((++polls & 4095) == 0) {
        const hipError_t e = hipStreamQuery(st);
        if (e == hipSuccess) idle_polls = 0;  // stream done: the report must be in flight
        else if (e != hipErrorNotReady) LSP_HIP(e);
      }
      __builtin_ia32_pause();
    }
    return __atomic_load_n(&h->nact, __ATOMIC_ACQUIRE);
  }
};

namespace {

void build_class_geometry(lsp_plan* pl) {
  const Plan& P = pl->p;
  const int d = P.d, n = P.n, b = P.opts.buffer_b;
  LSP_REQUIRE(b >= 1 && n - b - 1 >= 1, "buffer_b must satisfy 1 <= b <= n-2");
  pl->nclass = ipow(3, d);
  pl->geo.assign(pl->nclass, ClassGeom{});
  pl->maxF = 0;
  for (int c = 0; c < pl->nclass; ++c) {
    ClassGeom& g = pl->geo[c];
    int ct[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) ct[a] = (c / ipow(3, a)) % 3;
    int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
    bool interior = true;
    for (int a = 0; a < d; ++a) {
      if (ct[a] == 0) { lo[a] = 0; cnt[a] = 2; g.flo[a] = b + 1; g.fsz[a] = n - b - 1; interior = false; }
      else if (ct[a] == 1) { lo[a] = -1; cnt[a] = 3; g.flo[a] = -n + 1; g.fsz[a] = 2 * n - 1; }
      else { lo[a] = -1; cnt[a] = 2; g.flo[a] = -n + 1; g.fsz[a] = n - b - 1; interior = false; }
    }
    for (int a = d; a < 3; ++a) { g.flo[a] = 0; g.fsz[a] = 1; }
    g.s = cnt[0] * cnt[1] * cnt[2];
    for (int s = 0; s < g.s; ++s) {
      int r = s;
      for (int a = 0; a < 3; ++a) {
        g.off[s][a] = a < d ? lo[a] + r % cnt[a] : 0;
        r /= cnt[a];
      }
    }
    g.F = 1;
    for (int a = 0; a < d; ++a) g.F *= g.fsz[a];
    g.interior = interior ? 1 : 0;
    LSP_REQUIRE(g.F < (1LL << 31), "far set too large for 32-bit column indices");
    pl->maxF = std::max(pl->maxF, g.F);
  }
  // about 1024 far-set columns per Gram workgroup (measured on 2D n = 256:
  // 512 and 4096 columns per workgroup were 1.4x and 2.2x slower)
  long long nb = (pl->maxF + 1023) / 1024;
  pl->gram_blocks = (int)std::max<long long>(1, std::min<long long>(nb, 512));
}

// Gauss-Legendre nodes and weights on [0, 1] (Newton iteration on the
// Legendre recurrence from the Chebyshev-like initial guesses).
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  const double pi = 3.14159265358979323846;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2 / ((1 - z^2) P'^2), halved for [0, 1]
  }
}

// k_0 as the integral of G over the grid cell [-h/2, h/2]^d.  Over the part
// of the cell seen through a face (an edge in 2D) at distance h/2, the radial
// integral has a closed form at each distance rho = |(h/2, y[, z])| to the
// face: 2D int_0^rho G r dr = i rho H1(w rho) / (4 w) - 1 / (2 pi w^2),
// 3D (e^{i w rho}(1 - i w rho) - 1) / (4 pi w^2); the solid-angle element
// is (h/2) / rho^d, and the 4 edges x 2 halves (2D) / 6 faces x 4 quarters
// (3D) are equal by symmetry.  Gauss-Legendre on the smooth rest.
double2 cell_self_term(double h, double omega, int d) {
  const double pi = 3.14159265358979323846, a = 0.5 * h;
  std::vector<double> x, w;
  gauss_legendre01(32, x, w);
  double re = 0.0, im = 0.0;
  if (d == 2) {
    for (size_t i = 0; i < x.size(); ++i) {
      const double y = a * x[i], rho = std::sqrt(a * a + y * y), z = omega * rho;
      const double j1 = std::cyl_bessel_j(1.0, z), y1 = std::cyl_neumann(1.0, z);
      const double jac = a / (rho * rho) * a * w[i];
      re += (-rho * y1 / (4.0 * omega) - 1.0 / (2.0 * pi * omega * omega)) * jac;
      im += rho * j1 / (4.0 * omega) * jac;
    }
    return make_double2(8.0 * re, 8.0 * im);
  }
  for (size_t i = 0; i < x.size(); ++i)
    for (size_t j = 0; j < x.size(); ++j) {
      const double y = a * x[i], zz = a * x[j];
      const double rho = std::sqrt(a * a + y * y + zz * zz), t = omega * rho;
      const double jac = a / (rho * rho * rho) * a * a * w[i] * w[j] / (4.0 * pi);
      if (omega == 0.0) {  // the radial integral of 1/(4 pi r) r^2: rho^2 / 2
        re += 0.5 * rho * rho * jac;
      } else {
        const double c = std::cos(t), sn = std::sin(t);
        re += (c + t * sn - 1.0) * jac / (omega * omega);
        im += (sn - t * c) * jac / (omega * omega);
      }
    }
  return make_double2(24.0 * re, 24.0 * im);
}

// e^{-x} Ei(x), x > 0: the series gamma + ln x + sum_{k>=1} x^k / (k k!)
// (A&S 5.1.10; every term positive) up to x = 50, beyond it the asymptotic
// series sum_k k! / x^{k+1} (A&S 5.1.51) to its smallest term.
double expei(double x) {
  if (x <= 50.0) {
    double term = 1.0, sum = 0.0;
    for (int k = 1; k < 500; ++k) {
      term *= x / k;  // x^k / k!
      const double add = term / k;
      sum += add;
      if (add < 1e-18 * sum) break;
    }
    return std::exp(-x) * (0.57721566490153286061 + std::log(x) + sum);
  }
  double term = 1.0 / x, sum = term;
  for (int k = 1; k < 400; ++k) {
    const double next = term * k / x;
    if (next >= term || next < 1e-18 * sum) break;
    term = next;
    sum += term;
  }
  return sum;
}

// Dawson's integral F(z) = e^{-z^2} int_0^z e^{t^2} dt = int_0^z e^{-u (2z - u)} du
// (t = z - u), by Gauss-Legendre on 8 panels of [0, min(z, 40 / z)]
// (beyond, the integrand is below e^{-40}).
double dawson(double z) {
  if (z <= 0.0) return 0.0;
  std::vector<double> x, w;
  gauss_legendre01(32, x, w);
  const double U = std::min(z, 40.0 / z), panel = U / 8.0;
  double sum = 0.0;
  for (int p = 0; p < 8; ++p)
    for (size_t i = 0; i < x.size(); ++i) {
      const double u = panel * (p + x[i]);
      sum += w[i] * std::exp(-u * (2.0 * z - u));
    }
  return sum * panel;
}

// k_0 as a one-point correction of the trapezoid rule fitted to a unit
// Gaussian probe g of width sigma = max(0.05, 3h): k_0 = int G g - sum_{t != 0}
// h^d G(h t) g(h t), so the corrected rule integrates G g exactly; the
// integral in closed form (2D: Re = -sigma^2 e^{-x} Ei(x) / 2, Im = (pi/2)
// sigma^2 e^{-x}, x = w^2 sigma^2 / 2; 3D: Re = sigma^2 - sqrt(2) w sigma^3
// F(z), Im = sqrt(pi/2) w sigma^3 e^{-z^2}, z = w sigma / sqrt(2)), the
// lattice sum over 0 < |t| h <= 12 sigma, one representative per class of
// signed permutations, times the class size.  Cached per (h, w, d).
double2 fitted_self_term(double h, double omega, int d) {
  static std::mutex mu;
  static std::map<std::tuple<double, double, int>, double2> cache;
  const auto key = std::make_tuple(h, omega, d);
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  const double pi = 3.14159265358979323846;
  const double sigma = std::max(0.05, 3.0 * h), a = 0.5 / (sigma * sigma), R = 12.0 * sigma;
  const double s2 = sigma * sigma;
  double ire, iim;
  if (d == 2) {
    const double x = 0.5 * omega * omega * s2;
    ire = -0.5 * s2 * expei(x);
    iim = 0.5 * pi * s2 * std::exp(-x);
  } else {
    const double z = omega * sigma / std::sqrt(2.0);
    ire = s2 - std::sqrt(2.0) * omega * s2 * sigma * dawson(z);
    iim = std::sqrt(0.5 * pi) * omega * s2 * sigma * std::exp(-z * z);
  }
  const int m = (int)std::floor(R / h);
  double sre = 0.0, sim = 0.0;
  for (int t1 = 1; t1 <= m; ++t1)
    for (int t2 = 0; t2 <= t1; ++t2)
      for (int t3 = 0; t3 <= (d == 3 ? t2 : 0); ++t3) {
        const double r = h * std::sqrt((double)t1 * t1 + (double)t2 * t2 + (double)t3 * t3);
        if (r > R) continue;
        double mult;
        if (d == 2) {
          mult = (t2 == 0 || t2 == t1) ? 4.0 : 8.0;
        } else {
          const int perms = (t1 == t2 && t2 == t3) ? 1 : ((t1 == t2 || t2 == t3) ? 3 : 6);
          mult = perms * (double)(1 << (1 + (t2 > 0) + (t3 > 0)));
        }
        const double gw = mult * std::exp(-a * r * r);
        if (d == 2) {  // G = (i/4)(J0 + i Y0)
          const double z = omega * r;
          sre += gw * (-0.25 * std::cyl_neumann(0.0, z));
          sim += gw * (0.25 * std::cyl_bessel_j(0.0, z));
        } else {
          const double c = std::cos(omega * r), sn = std::sin(omega * r), inv = 1.0 / (4.0 * pi * r);
          sre += gw * c * inv;
          sim += gw * sn * inv;
        }
      }
  const double hd = d == 2 ? h * h : h * h * h;
  const double2 k0 = make_double2(ire - hd * sre, iim - hd * sim);
  std::lock_guard<std::mutex> lock(mu);
  cache[key] = k0;
  return k0;
}

double2 self_term_host(double h, double omega, int d, int mode) {
  const double pi = 3.14159265358979323846;
  if (mode == 1) return cell_self_term(h, omega, d);
  if (mode == 2) return fitted_self_term(h, omega, d);
  if (d == 2) {
    double rho = h / std::sqrt(pi);
    double z = omega * rho;
    double j1 = std::cyl_bessel_j(1.0, z), y1 = std::cyl_neumann(1.0, z);
    // (i pi rho / (2 w)) (J1 + i Y1) - 1/w^2
    double s = pi * rho / (2.0 * omega);
    return make_double2(-s * y1 - 1.0 / (omega * omega), s * j1);
  }
  double rho = h * std::cbrt(3.0 / (4.0 * pi));
  if (omega == 0.0) return make_double2(0.5 * rho * rho, 0.0);  // the Laplace limit
  double z = omega * rho;
  double c = std::cos(z), sn = std::sin(z);
  // (e^{iz}(1 - iz) - 1) / w^2
  double re = c + z * sn - 1.0, im = sn - z * c;
  return make_double2(re / (omega * omega), im / (omega * omega));
}

// The tile table of (n, d, precision) from a cache file written by
// lsp_plan_save_tiles; false when absent, malformed or of another level count.
bool read_tile_line(const std::string& path, const Plan& P, std::vector<int>& tiles) {
  std::ifstream in(path);
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {
    std::istringstream ss(line);
    int n = 0, d = 0, prec = -1, nl = 0;
    if (!(ss >> n >> d >> prec >> nl)) continue;
    if (n != P.n || d != P.d || prec != P.opts.precision || nl != P.nlevels) continue;
    std::vector<int> t(nl);
    bool ok = true;
    for (int l = 0; l < nl && ok; ++l) ok = (ss >> t[l]) && (t[l] == 32 || t[l] == 64 || t[l] == 128);
    if (ok) {
      tiles = t;
      found = true;
    }
  }
  return found;
}

template <typename T>
FftPlanDev<T> make_fft_plan(const Plan& P, const cplx<T>* tw, const cplx<T>* spec) {
  FftPlanDev<T> f{};
  f.n = P.n; f.d = P.d; f.L = P.L; f.N = P.N;
  bool has3 = false;
  for (int r : P.radices) has3 = has3 || r == 3;
  if (!has3) f.ept = 8;
  else {
    int c2 = 0, L = P.L;
    while (L % 2 == 0) { L /= 2; ++c2; }
    f.ept = c2 >= 2 ? 12 : 6;
  }
  long long Ld = 1;
  for (int a = 0; a < P.d; ++a) Ld *= P.L;
  f.wstride = Ld;
  // 2D work rows padded by 16 elements (n rows of L + 16 fit in L^2 for n >= 16)
  f.lr = P.d == 2 && P.n >= 16 ? P.L + 16 : P.L;
  f.rad.npass = (int)P.radices.size();
  for (int i = 0; i < f.rad.npass; ++i) f.rad.r[i] = P.radices[i];
  // the n-point transforms of the K-matvec: n = 2^a 3^b
  {
    int r = P.n, a = 0, b = 0;
    while (r % 2 == 0) { r /= 2; ++a; }
    while (r % 3 == 0) { r /= 3; ++b; }
    std::vector<int> rad;
    if (b == 0) {
      f.hept = a >= 3 ? 8 : P.n;
      if (a % 3) rad.push_back(1 << (a % 3));
      for (int k = 0; k < a / 3; ++k) rad.push_back(8);
    } else {
      f.hept = 3 << std::min(a, 2);
      for (int k = 0; k < a / 2; ++k) rad.push_back(4);
      if (a % 2) rad.push_back(2);
      for (int k = 0; k < b; ++k) rad.push_back(3);
    }
    LSP_REQUIRE(r == 1 && (int)rad.size() <= 16, "n must be 2^a 3^b");
    f.hrad.npass = (int)rad.size();
    for (int i = 0; i < f.hrad.npass; ++i) f.hrad.r[i] = rad[i];
  }
  f.tw = tw; f.spec = spec;
  return f;
}

// radices for lengths containing a factor 3 are 4s, a 2, then 3s (EPT 12 or 6)
void fix_radices(Plan& P) {
  bool has3 = false;
  for (int r : P.radices) has3 = has3 || r == 3;
  if (!has3) return;
  int L = P.L, c2 = 0, c3 = 0;
  while (L % 2 == 0) { L /= 2; ++c2; }
  while (L % 3 == 0) { L /= 3; ++c3; }
  std::vector<int> rad;
  int t = c2;
  while (t >= 2) { rad.push_back(4); t -= 2; }
  if (t == 1) rad.push_back(2);
  for (int k = 0; k < c3; ++k) rad.push_back(3);
  P.radices = rad;
}

// z = Q v (the class stencils, or a general domain's per-point rows)
template <typename Cx>
void apply_Q(lsp_problem* pb, Cx* z, const double2* v, int nrhs) {
  const Plan& P = pb->plan->p;
  if (P.general)
    launch_applyQ_general<Cx>(z, v, pb->d.alpha_pad, pb->d.ptab, pb->d.balpha, P.n, P.d, P.N, nrhs, pb->st);
  else
    launch_applyQ<Cx>(z, v, pb->d.alpha_pad, P.n, P.d, P.N, nrhs, pb->st);
}

void apply_precond(lsp_problem* pb, const SolvePtrs& s, int nrhs, const double2* v, double2* out) {
  const Plan& P = pb->plan->p;
  hipStream_t st = pb->st;
  if (pb->precision == LSP_FP64) {
    apply_Q<double2>(pb, (double2*)s.zq, v, nrhs);
    MfDev<double> mf{(double2*)pb->d.F, (double2*)pb->d.Dinv, pb->d.fronts, pb->d.idx, pb->d.gpos, pb->d.cpos, pb->d.Mval, pb->d.perm,
                     pb->d.pivstat, (double2*)pb->d.Gop};
    const SweepBufs<double> sb{(double2*)s.ybuf, (double2*)s.pbuf, P.bsweep_ystride, (double2*)s.xpm};
    mf_solve<double>(mf, P, nrhs, (const double2*)s.zq, out, (double2*)s.vbuf, sb, st, pb->take_form_wait(), nullptr);
  } else {
    apply_Q<float2>(pb, (float2*)s.zq, v, nrhs);
    MfDev<float> mf{(float2*)pb->d.F, (float2*)pb->d.Dinv, pb->d.fronts, pb->d.idx, pb->d.gpos, pb->d.cpos, pb->d.Mval, pb->d.perm,
                    pb->d.pivstat, (float2*)pb->d.Gop};
    // the backward sweeps also store the solution widened into out
    const SweepBufs<float> sb{(float2*)s.ybuf, (float2*)s.pbuf, P.bsweep_ystride, (float2*)s.xpm};
    mf_solve<float>(mf, P, nrhs, (const float2*)s.zq, (float2*)s.xs, (float2*)s.vbuf, sb, st, pb->take_form_wait(), out);
  }
}

void solve_M(lsp_problem* pb, const SolvePtrs& s, int nrhs, const double2* z, double2* x) {
  const Plan& P = pb->plan->p;
  hipStream_t st = pb->st;
  if (pb->precision == LSP_FP64) {
    MfDev<double> mf{(double2*)pb->d.F, (double2*)pb->d.Dinv, pb->d.fronts, pb->d.idx, pb->d.gpos, pb->d.cpos, pb->d.Mval, pb->d.perm,
                     pb->d.pivstat, (double2*)pb->d.Gop};
    const SweepBufs<double> sb{(double2*)s.ybuf, (double2*)s.pbuf, P.bsweep_ystride, (double2*)s.xpm};
    mf_solve<double>(mf, P, nrhs, z, x, (double2*)s.vbuf, sb, st, pb->take_form_wait(), nullptr);
  } else {
    launch_narrow((float2*)s.zq, z, (long long)nrhs * P.N, st);
    MfDev<float> mf{(float2*)pb->d.F, (float2*)pb->d.Dinv, pb->d.fronts, pb->d.idx, pb->d.gpos, pb->d.cpos, pb->d.Mval, pb->d.perm,
                    pb->d.pivstat, (float2*)pb->d.Gop};
    const SweepBufs<float> sb{(float2*)s.ybuf, (float2*)s.pbuf, P.bsweep_ystride, (float2*)s.xpm};
    mf_solve<float>(mf, P, nrhs, (const float2*)s.zq, (float2*)s.xs, (float2*)s.vbuf, sb, st, pb->take_form_wait(), x);
  }
}

// y = x + K(w2m .* x) (op) or K x, in the given precision; on a general
// domain y is restricted to Omega (zero outside)
void apply_conv(lsp_problem* pb, const SolvePtrs& s, int nrhs, int precision, const double2* x, double2* y, bool op,
                const double* w2m) {
  if (precision == LSP_MIXED)
    kmatvec<float>(pb->fp32, nrhs, x, y, w2m, op, (float2*)s.W, pb->st, pb->d.dmask);
  else
    kmatvec<double>(pb->fp64, nrhs, x, y, w2m, op, (double2*)s.W, pb->st, pb->d.dmask);
}

void check_ws(const lsp_problem* pb, int nrhs, bool krylov, void* ws, size_t bytes) {
  LSP_REQUIRE(nrhs >= 1 && nrhs <= pb->plan->p.max_nrhs, "nrhs out of range for this plan");
  LSP_REQUIRE(ws != nullptr, "null workspace");
  size_t need = layout_solve(pb->plan->p, nrhs, pb->plan->p.opts.restart, krylov, nullptr, nullptr);
  LSP_REQUIRE(bytes >= need, "solve workspace too small");
}

}  // namespace

extern "C" {

const char* lsp_status_string(lsp_status s) {
  switch (s) {
    case LSP_OK: return "ok";
    case LSP_ERR_ARG: return "invalid argument";
    case LSP_ERR_OOM: return "out of memory";
    case LSP_ERR_HIP: return "HIP runtime error";
    case LSP_ERR_STATE: return "invalid call order";
    case LSP_ERR_SINGULAR: return "singular pivot";
    case LSP_ERR_NOCONV: return "GMRES did not converge";
  }
  return "unknown status";
}

void lsp_last_error(char* buf, size_t len) {
  if (!buf || len == 0) return;
  size_t k = std::min(len - 1, g_last_error.size());
  std::memcpy(buf, g_last_error.data(), k);
  buf[k] = 0;
}

lsp_status lsp_options_default(lsp_options* o) {
  if (!o) return fail(LSP_ERR_ARG, "null options");
  o->tol = 1e-8;
  o->restart = 30;
  o->max_iters = 1000;
  o->precision = LSP_FP64;
  o->buffer_b = 2;
  o->leaf = 0;
  o->panel = 0;
  o->dense_sweeps = 1;
  o->blocked_sweeps = 1;
  o->self_term = 0;
  o->equation = LSP_HELMHOLTZ;
  o->tile_cache = nullptr;
  return LSP_OK;
}

static lsp_status plan_create_impl(int n, int d, int max_nrhs, const lsp_options* opts, const unsigned char* mask,
                            int sketch_cols, lsp_plan** out) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(out != nullptr, "null plan pointer");
    *out = nullptr;
    lsp_options o;
    if (opts) o = *opts; else lsp_options_default(&o);
    LSP_REQUIRE(o.tol > 0 && std::isfinite(o.tol), "tol must be positive");
    LSP_REQUIRE(o.restart >= 1 && o.restart < kMaxVec, "restart must be in [1, 31]");
    LSP_REQUIRE(o.max_iters >= 1, "max_iters must be >= 1");
    LSP_REQUIRE(o.precision == LSP_FP64 || o.precision == LSP_MIXED, "unknown precision");
    LSP_REQUIRE(o.panel == 0 || o.panel == kNbMax, "panel must be 0 (auto) or 32");
    LSP_REQUIRE(o.dense_sweeps >= 0 && o.dense_sweeps <= 2, "dense_sweeps must be 0, 1 or 2");
    LSP_REQUIRE(o.blocked_sweeps >= 0 && o.blocked_sweeps <= 2, "blocked_sweeps must be 0, 1 or 2");
    LSP_REQUIRE(o.self_term >= 0 && o.self_term <= 2, "self_term must be 0, 1 or 2");
    LSP_REQUIRE(o.equation == LSP_HELMHOLTZ || o.equation == LSP_LAPLACE, "unknown equation");
    LSP_REQUIRE(o.equation == LSP_HELMHOLTZ || d == 3, "the Laplace equation is three-dimensional (d must be 3)");
    const std::string cache = o.tile_cache ? o.tile_cache : "";
    o.tile_cache = nullptr;  // the plan keeps no pointer into the caller's memory
    std::unique_ptr<lsp_plan> pl(new lsp_plan());
    build_plan(pl->p, n, d, max_nrhs, o);
    if (mask) {
      LSP_REQUIRE(o.equation == LSP_HELMHOLTZ, "general domains are for the Helmholtz equation");
      build_general(pl->p, mask, sketch_cols > 0 ? sketch_cols : 2 * ipow(3, d));
    }
    fix_radices(pl->p);
    build_class_geometry(pl.get());
    if (!cache.empty()) {
      std::vector<int> t;
      if (read_tile_line(cache, pl->p, t)) pl->p.level_tile = t;
    }
    *out = pl.release();
    return LSP_OK;
  });
}

lsp_status lsp_plan_create(int n, int d, int max_nrhs, const lsp_options* opts, lsp_plan** out) {
  return plan_create_impl(n, d, max_nrhs, opts, nullptr, 0, out);
}

lsp_status lsp_plan_create_general(int n, int d, int max_nrhs, const lsp_options* opts, const unsigned char* mask,
                                   int sketch_cols, lsp_plan** out) {
  if (!mask) return fail(LSP_ERR_ARG, "null domain mask");
  if (sketch_cols < 0) return fail(LSP_ERR_ARG, "sketch_cols must be >= 0");
  return plan_create_impl(n, d, max_nrhs, opts, mask, sketch_cols, out);
}

void lsp_plan_destroy(lsp_plan* plan) { delete plan; }

lsp_status lsp_plan_stats_get(const lsp_plan* plan, lsp_plan_stats* s) {
  if (!plan || !s) return fail(LSP_ERR_ARG, "null argument");
  const Plan& P = plan->p;
  s->n = P.n; s->d = P.d; s->N = P.N; s->L = P.L;
  s->nfronts = (int)P.fronts.size();
  s->nlevels = P.nlevels;
  s->max_front = P.max_front;
  s->max_pivots = P.max_p;
  s->factor_entries = P.factor_entries;
  s->front_entries = (double)P.front_elems;
  s->factor_flops = P.flops;
  s->sweep_entries = P.sweep_entries;
  s->update_flops = P.update_flops;
  s->panel_blocks = P.panel_blocks;
  const FactorSchedule fs = factor_schedule(P, P.opts.precision == LSP_FP64);
  s->fused_blocks = fs.fused_blocks;
  s->fused_update_flops = fs.fused_update_flops;
  s->dense_entries = P.dense_entries;
  s->dense_levels = P.dense_levels;
  s->blocked_levels = P.blocked_levels;
  s->blocked_entries = P.blocked_entries;
  s->chain_entries = P.chain_entries;
  s->blocked_panel_entries = P.blocked_panel_entries;
  s->trsm_flops = fs.trsm_flops;
  s->assemble_entries = P.assemble_entries;
  s->mchain_levels = P.mchain_levels;
  s->mchain_entries = P.mchain_entries;
  s->pair_update_flops = fs.pair_update_flops;
  s->cross_update_flops = fs.cross_update_flops;
  s->mchain_pivots = P.mchain_pivots;
  s->mchain_rows = P.mchain_rows;
  s->mchain_child_rows = P.mchain_child_rows;
  s->domain_points = P.general ? P.domain_points : P.N;
  s->boundary_points = (int)P.bpts.size();
  s->sketch_cols = P.sketch_r;
  return LSP_OK;
}

lsp_status lsp_plan_get_tiles(const lsp_plan* plan, int* tiles, int cap) {
  if (!plan || (!tiles && cap > 0) || cap < 0) return fail(LSP_ERR_ARG, "null argument");
  const Plan& P = plan->p;
  for (int l = 0; l < std::min(cap, P.nlevels); ++l) tiles[l] = P.level_tile[l];
  return LSP_OK;
}

lsp_status lsp_plan_set_tiles(lsp_plan* plan, const int* tiles, int n) {
  if (!plan || !tiles) return fail(LSP_ERR_ARG, "null argument");
  Plan& P = plan->p;
  if (n != P.nlevels) return fail(LSP_ERR_ARG, "tile count must equal the number of levels");
  for (int l = 0; l < n; ++l)
    if (tiles[l] != 32 && tiles[l] != 64 && tiles[l] != 128) return fail(LSP_ERR_ARG, "tiles must be 32, 64 or 128");
  for (int l = 0; l < n; ++l) P.level_tile[l] = tiles[l];
  return LSP_OK;
}

lsp_status lsp_plan_save_tiles(const lsp_plan* plan, const char* path) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(plan != nullptr && path != nullptr, "null argument");
    const Plan& P = plan->p;
    std::vector<std::string> keep;
    {
      std::ifstream in(path);
      std::string line;
      while (std::getline(in, line)) {
        std::istringstream ss(line);
        int n = 0, d = 0, prec = -1;
        if (ss >> n >> d >> prec && n == P.n && d == P.d && prec == P.opts.precision) continue;
        if (!line.empty()) keep.push_back(line);
      }
    }
    std::ostringstream mine;
    mine << P.n << ' ' << P.d << ' ' << P.opts.precision << ' ' << P.nlevels;
    for (int t : P.level_tile) mine << ' ' << t;
    keep.push_back(mine.str());
    const std::string tmp = std::string(path) + ".tmp";
    {
      std::ofstream out(tmp, std::ios::trunc);
      for (const auto& l : keep) out << l << '\n';
      out.flush();
      LSP_REQUIRE(out.good(), std::string("cannot write the tile cache ") + tmp);
    }
    LSP_REQUIRE(std::rename(tmp.c_str(), path) == 0, std::string("cannot replace the tile cache ") + path);
    return LSP_OK;
  });
}

lsp_status lsp_plan_bytes(const lsp_plan* plan, int precision, int nrhs, size_t* problem_bytes, size_t* solve_bytes) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(plan != nullptr, "null plan");
    LSP_REQUIRE(precision == LSP_FP64 || precision == LSP_MIXED, "unknown precision");
    LSP_REQUIRE(nrhs >= 1 && nrhs <= plan->p.max_nrhs, "nrhs out of range");
    if (problem_bytes) *problem_bytes = layout_problem(plan, precision, nullptr, nullptr);
    if (solve_bytes) *solve_bytes = layout_solve(plan->p, nrhs, plan->p.opts.restart, true, nullptr, nullptr);
    return LSP_OK;
  });
}

static lsp_status setup_impl(const lsp_plan* plan, double omega, const double* m_dev, const double* R_dev, void* ws_dev,
                      size_t ws_bytes, void* stream, lsp_problem** out) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(out != nullptr, "null problem pointer");
    *out = nullptr;
    LSP_REQUIRE(plan != nullptr && m_dev != nullptr && ws_dev != nullptr, "null argument");
    LSP_REQUIRE(plan->p.general == (R_dev != nullptr),
                plan->p.general ? "a general-domain plan is set up with lsp_setup_general (sketch R)"
                                : "lsp_setup_general needs a plan from lsp_plan_create_general");
    if (plan->p.opts.equation == LSP_LAPLACE)
      LSP_REQUIRE(omega == 0.0, "omega must be 0 for the Laplace equation");
    else
      LSP_REQUIRE(std::isfinite(omega) && omega > 0, "omega must be positive and finite");
    const Plan& P = plan->p;
    const int prec = P.opts.precision;
    size_t need = layout_problem(plan, prec, nullptr, nullptr);
    LSP_REQUIRE(ws_bytes >= need, "problem workspace too small");
    std::unique_ptr<lsp_problem> pb(new lsp_problem());
    pb->plan = plan;
    pb->precision = prec;
    pb->omega = omega;
    pb->st = (hipStream_t)stream;
    LSP_HIP(hipGetDevice(&pb->device));
    char* base = (char*)align_up((size_t)ws_dev, 256);
    LSP_REQUIRE(ws_bytes - ((size_t)base - (size_t)ws_dev) >= need - 256, "problem workspace too small");
    layout_problem(plan, prec, base, &pb->d);
    hipStream_t st = pb->st;
    pb->take_events();
    LSP_HIP(hipEventRecord(pb->ev[lsp_problem::EV_SETUP0], st));

    // the plan's constant arrays (uploaded once per device)
    const PlanDev& pd = plan_device(plan, pb->device);
    pb->d.fronts = pd.fronts;
    pb->d.idx = pd.idx;
    pb->d.gpos = pd.gpos;
    pb->d.cpos = pd.cpos;
    pb->d.geo = pd.geo;
    pb->d.tw64 = pd.tw64;
    pb->d.tw32 = pd.tw32;
    pb->d.ptab = pd.ptab;
    pb->d.bpts = pd.bpts;
    pb->d.bslots = pd.bslots;
    pb->fp64 = make_fft_plan<double>(P, pb->d.tw64, pb->d.spec64);
    pb->fp32 = make_fft_plan<float>(P, pb->d.tw32, pb->d.spec32);

    // kernel table, medium, spectrum
    double h = 1.0 / P.n;
    launch_ktable(pb->d.ktab, P.n, P.d, omega, self_term_host(h, omega, P.d, P.opts.self_term), st);
    // w^2 m, or the potential V itself for the Laplace equation
    k_w2m(pb->d.w2m, m_dev, P.opts.equation == LSP_LAPLACE ? 1.0 : omega * omega, P.N, st);
    launch_embed(pb->d.E, pb->d.ktab, P.n, P.d, st);
    full_fft_forward<double>(pb->fp64, pb->d.E, st);
    launch_split_spectrum(pb->d.spec64, pb->d.spec32, pb->d.E, P.n, P.d, st);
    // stencils and the sparse matrix
    compute_stencils(pb->d.ktab, P.n, P.d, pb->d.geo, plan->nclass, plan->maxF, pb->d.partial, plan->gram_blocks,
                     pb->d.G, pb->d.U1, pb->d.alpha_pad, pb->d.C_pad, pb->d.sigma_pad, st);
    if (P.general) {
      // Section 4: T = (K w^2 m) R over Omega's columns, the K products in
      // batches of kSketchBatch sketch columns (in place), then the
      // boundary points' stencils
      launch_domain_mask(pb->d.dmask, pb->d.ptab, P.N, st);
      for (int c = 0; c < P.sketch_r; ++c)
        launch_sketch_widen(pb->d.T + (size_t)c * P.N, R_dev + (size_t)c * P.N, pb->d.ptab, P.N, st);
      for (int c0 = 0; c0 < P.sketch_r; c0 += kSketchBatch) {
        const int g = std::min(kSketchBatch, P.sketch_r - c0);
        double2* Tc = pb->d.T + (size_t)c0 * P.N;
        kmatvec<double>(pb->fp64, g, Tc, Tc, pb->d.w2m, false, pb->d.Tw, st);
      }
      launch_bnd_stencils(pb->d.T, P.sketch_r, P.N, pb->d.bpts, pb->d.bslots, (int)P.bpts.size(), P.n, P.d,
                          pb->d.balpha, pb->d.bsigma, st);
      launch_assemble_general(pb->d.Mval, pb->d.alpha_pad, pb->d.C_pad, pb->d.w2m, pb->d.ptab, pb->d.balpha, P.n,
                              P.d, P.N, st);
    } else {
      launch_assemble(pb->d.Mval, pb->d.alpha_pad, pb->d.C_pad, pb->d.w2m, P.n, P.d, P.N, st);
    }
    LSP_HIP(hipEventRecord(pb->ev[lsp_problem::EV_SETUP1], st));
    *out = pb.release();
    return LSP_OK;
  });
}

lsp_status lsp_setup(const lsp_plan* plan, double omega, const double* m_dev, void* ws_dev, size_t ws_bytes,
                     void* stream, lsp_problem** out) {
  return setup_impl(plan, omega, m_dev, nullptr, ws_dev, ws_bytes, stream, out);
}

lsp_status lsp_setup_general(const lsp_plan* plan, double omega, const double* m_dev, const double* R_dev,
                             void* ws_dev, size_t ws_bytes, void* stream, lsp_problem** out) {
  if (!R_dev) return fail(LSP_ERR_ARG, "null sketch matrix");
  return setup_impl(plan, omega, m_dev, R_dev, ws_dev, ws_bytes, stream, out);
}

lsp_status lsp_self_term(double h, double omega, int d, int mode, double* k0) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(k0 != nullptr, "null output");
    LSP_REQUIRE(d == 2 || d == 3, "d must be 2 or 3");
    LSP_REQUIRE(mode >= 0 && mode <= 2, "self_term must be 0, 1 or 2");
    LSP_REQUIRE(h > 0 && std::isfinite(h) && omega >= 0 && std::isfinite(omega), "invalid h or omega");
    LSP_REQUIRE(d == 3 || omega > 0, "omega = 0 (the Laplace kernel) is three-dimensional");
    const double2 v = self_term_host(h, omega, d, mode);
    k0[0] = v.x;
    k0[1] = v.y;
    return LSP_OK;
  });
}

lsp_status lsp_field_bytes(const lsp_plan* plan, int npts, size_t* bytes) {
  if (!plan || !bytes) return fail(LSP_ERR_ARG, "null argument");
  if (npts < 1) return fail(LSP_ERR_ARG, "npts must be >= 1");
  *bytes = (size_t)field_chunks(plan->p.N) * 16 * (size_t)npts * sizeof(double2) + 256;
  return LSP_OK;
}

static lsp_status field_impl(int mode, lsp_problem* pb, int nrhs, const void* u, const void* uI, int npts,
                             const double* pts, void* out, void* ws, size_t bytes) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb && u && uI && pts && out && ws, "null argument");
    LSP_REQUIRE(nrhs >= 1 && npts >= 1, "nrhs and npts must be >= 1");
    const Plan& P = pb->plan->p;
    LSP_REQUIRE(P.opts.equation == LSP_HELMHOLTZ, "field evaluation is for the Helmholtz equation");
    size_t need = 0;
    lsp_field_bytes(pb->plan, npts, &need);
    LSP_REQUIRE(bytes >= need, "field workspace too small");
    const double2 k0 = self_term_host(1.0 / P.n, pb->omega, P.d, P.opts.self_term);
    field_eval(mode, (const double2*)u, (const double2*)uI, pb->d.w2m, pts, npts, nrhs, P.n, P.d, pb->omega, k0,
               (double2*)align_up((size_t)ws, 256), (double2*)out, pb->st);
    return LSP_OK;
  });
}

lsp_status lsp_exterior_field(lsp_problem* pb, int nrhs, const void* u, const void* uI, int npts,
                              const double* points, void* out, void* ws, size_t bytes) {
  return field_impl(0, pb, nrhs, u, uI, npts, points, out, ws, bytes);
}

lsp_status lsp_far_field(lsp_problem* pb, int nrhs, const void* u, const void* uI, int ndirs, const double* dirs,
                         void* out, void* ws, size_t bytes) {
  return field_impl(1, pb, nrhs, u, uI, ndirs, dirs, out, ws, bytes);
}

lsp_status lsp_get_boundary_stencils(lsp_problem* pb, int* points, double* alpha, double* sigma) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb != nullptr, "null problem");
    const Plan& P = pb->plan->p;
    LSP_REQUIRE(P.general, "not a general-domain problem");
    const size_t nb = P.bpts.size(), S = kMaxStencil;
    if (points && nb) std::memcpy(points, P.bpts.data(), nb * sizeof(int));
    if (alpha && nb)
      LSP_HIP(hipMemcpyAsync(alpha, pb->d.balpha, nb * S * sizeof(double2), hipMemcpyDeviceToHost, pb->st));
    if (sigma && nb)
      LSP_HIP(hipMemcpyAsync(sigma, pb->d.bsigma, nb * S * sizeof(double), hipMemcpyDeviceToHost, pb->st));
    LSP_HIP(hipStreamSynchronize(pb->st));
    return LSP_OK;
  });
}

void lsp_problem_destroy(lsp_problem* pb) { delete pb; }

lsp_status lsp_factor(lsp_problem* pb) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb != nullptr, "null problem");
    const Plan& P = pb->plan->p;
    if (P.dense_levels + P.blocked_levels > 0 && !pb->fs.aux) {
      int cur = 0;
      LSP_HIP(hipGetDevice(&cur));
      if (cur != pb->device) LSP_HIP(hipSetDevice(pb->device));
      try {
        pb->fs = lsp_problem::form_pool().get(pb->device, pb->st);
      } catch (...) {
        if (cur != pb->device) (void)hipSetDevice(cur);
        throw;
      }
      if (cur != pb->device) LSP_HIP(hipSetDevice(cur));
    }
    const FormStream* fsp = pb->fs.aux ? &pb->fs : nullptr;
    pb->form_pending = fsp != nullptr;
    LSP_HIP(hipEventRecord(pb->ev[lsp_problem::EV_FACTOR0], pb->st));
    if (pb->precision == LSP_FP64) {
      MfDev<double> mf{(double2*)pb->d.F, (double2*)pb->d.Dinv, pb->d.fronts, pb->d.idx, pb->d.gpos, pb->d.cpos, pb->d.Mval, pb->d.perm,
                       pb->d.pivstat, (double2*)pb->d.Gop};
      mf_factor<double>(mf, P, pb->st, fsp);
    } else {
      MfDev<float> mf{(float2*)pb->d.F, (float2*)pb->d.Dinv, pb->d.fronts, pb->d.idx, pb->d.gpos, pb->d.cpos, pb->d.Mval, pb->d.perm,
                      pb->d.pivstat, (float2*)pb->d.Gop};
      mf_factor<float>(mf, P, pb->st, fsp);
    }
    // smallest pivot ratio over the diagonal blocks (a NaN counts as -1), reported
    // into the pinned control block
    pb->ensure_host(1);
    k_min_report(pb->d.pivstat, (long long)P.panel_blocks, lsp_problem::ctl_view(pb->ctl_dev, pb->host_cap),
                 ++pb->ctl_tag, pb->st);
    LSP_HIP(hipEventRecord(pb->ev[lsp_problem::EV_FACTOR1], pb->st));
    pb->factor_timed = true;
    pb->wait_ctl(pb->ctl_tag);
    const double mn = lsp_problem::ctl_view(pb->ctl_host, pb->host_cap).hdr->value;
    pb->min_pivot_ratio = mn;
    const double eps = pb->precision == LSP_FP64 ? 2.220446049250313e-16 : 1.1920928955078125e-07;
    if (!(mn > 64.0 * eps)) {
      pb->factored = false;
      throw Error(LSP_ERR_SINGULAR, "zero pivot in the multifrontal factorisation");
    }
    pb->factored = true;
    return LSP_OK;
  });
}

lsp_status lsp_apply_op(lsp_problem* pb, int nrhs, int precision, const void* x, void* y, void* ws, size_t bytes) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb && x && y, "null argument");
    LSP_REQUIRE(precision == LSP_FP64 || precision == LSP_MIXED, "unknown precision");
    check_ws(pb, nrhs, false, ws, bytes);
    SolvePtrs s;
    layout_solve(pb->plan->p, nrhs, pb->plan->p.opts.restart, false, (void*)align_up((size_t)ws, 256), &s);
    apply_conv(pb, s, nrhs, precision, (const double2*)x, (double2*)y, true, pb->d.w2m);
    return LSP_OK;
  });
}

lsp_status lsp_apply_K(lsp_problem* pb, int nrhs, int precision, const void* x, void* y, void* ws, size_t bytes) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb && x && y, "null argument");
    LSP_REQUIRE(precision == LSP_FP64 || precision == LSP_MIXED, "unknown precision");
    check_ws(pb, nrhs, false, ws, bytes);
    SolvePtrs s;
    layout_solve(pb->plan->p, nrhs, pb->plan->p.opts.restart, false, (void*)align_up((size_t)ws, 256), &s);
    apply_conv(pb, s, nrhs, precision, (const double2*)x, (double2*)y, false, nullptr);
    return LSP_OK;
  });
}

lsp_status lsp_apply_op_noalloc(lsp_problem* pb, int nrhs, int precision, const void* x, void* y) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb && x && y, "null argument");
    LSP_REQUIRE(precision == LSP_FP64 || precision == LSP_MIXED, "unknown precision");
    LSP_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    const Plan& P = pb->plan->p;
    long long Ld = 1;
    for (int a = 0; a < P.d; ++a) Ld *= P.L;
    const size_t esz = precision == LSP_MIXED ? sizeof(float2) : sizeof(double2);
    const size_t need = (size_t)nrhs * (size_t)Ld * esz;
    if (need > kStaticScratchBytes)
      throw Error(LSP_ERR_ARG, "lsp_apply_op_noalloc: the FFT work array needs " + std::to_string(need) +
                                   " bytes (nrhs (2n)^d elements), more than the " +
                                   std::to_string(kStaticScratchBytes) + "-byte static scratch");
    // the device's scratch address (looked up on the first call per device);
    // the kernels overwrite every element of it they read, so nothing is cleared
    void* W = static_scratch(pb->device);
    if (precision == LSP_MIXED)
      kmatvec<float>(pb->fp32, nrhs, (const double2*)x, (double2*)y, pb->d.w2m, true, (float2*)W, pb->st,
                     pb->d.dmask);
    else
      kmatvec<double>(pb->fp64, nrhs, (const double2*)x, (double2*)y, pb->d.w2m, true, (double2*)W, pb->st,
                      pb->d.dmask);
    return LSP_OK;
  });
}

lsp_status lsp_apply_Q(lsp_problem* pb, int nrhs, const void* x, void* y) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb && x && y, "null argument");
    LSP_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    apply_Q<double2>(pb, (double2*)y, (const double2*)x, nrhs);
    return LSP_OK;
  });
}

lsp_status lsp_solve_M(lsp_problem* pb, int nrhs, const void* z, void* x, void* ws, size_t bytes) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb && z && x, "null argument");
    if (!pb->factored) throw Error(LSP_ERR_STATE, "lsp_factor has not succeeded on this problem");
    check_ws(pb, nrhs, false, ws, bytes);
    SolvePtrs s;
    layout_solve(pb->plan->p, nrhs, pb->plan->p.opts.restart, false, (void*)align_up((size_t)ws, 256), &s);
    solve_M(pb, s, nrhs, (const double2*)z, (double2*)x);
    return LSP_OK;
  });
}

lsp_status lsp_apply_precond(lsp_problem* pb, int nrhs, const void* v, void* x, void* ws, size_t bytes) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb && v && x, "null argument");
    if (!pb->factored) throw Error(LSP_ERR_STATE, "lsp_factor has not succeeded on this problem");
    check_ws(pb, nrhs, false, ws, bytes);
    SolvePtrs s;
    layout_solve(pb->plan->p, nrhs, pb->plan->p.opts.restart, false, (void*)align_up((size_t)ws, 256), &s);
    apply_precond(pb, s, nrhs, (const double2*)v, (double2*)x);
    return LSP_OK;
  });
}

lsp_status lsp_get_kernel_table(lsp_problem* pb, void* k_dev) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb && k_dev, "null argument");
    const Plan& P = pb->plan->p;
    long long n1d = 1;
    for (int a = 0; a < P.d; ++a) n1d *= P.n + 1;
    LSP_HIP(hipMemcpyAsync(k_dev, pb->d.ktab, n1d * sizeof(double2), hipMemcpyDeviceToDevice, pb->st));
    LSP_HIP(hipStreamSynchronize(pb->st));
    return LSP_OK;
  });
}

lsp_status lsp_get_stencils(lsp_problem* pb, double* alpha, double* sigma, double* C) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb != nullptr, "null problem");
    const int nc = pb->plan->nclass, S = kMaxStencil;
    if (alpha)
      LSP_HIP(hipMemcpyAsync(alpha, pb->d.alpha_pad, (size_t)nc * S * sizeof(double2), hipMemcpyDeviceToHost, pb->st));
    if (C) LSP_HIP(hipMemcpyAsync(C, pb->d.C_pad, (size_t)nc * S * sizeof(double2), hipMemcpyDeviceToHost, pb->st));
    if (sigma)
      LSP_HIP(hipMemcpyAsync(sigma, pb->d.sigma_pad, (size_t)nc * S * sizeof(double), hipMemcpyDeviceToHost, pb->st));
    LSP_HIP(hipStreamSynchronize(pb->st));
    return LSP_OK;
  });
}

lsp_status lsp_get_matrix(lsp_problem* pb, void* mval) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb && mval, "null argument");
    const Plan& P = pb->plan->p;
    size_t bytes = (size_t)P.N * (P.d == 2 ? 9 : 27) * sizeof(double2);
    LSP_HIP(hipMemcpyAsync(mval, pb->d.Mval, bytes, hipMemcpyDeviceToDevice, pb->st));
    LSP_HIP(hipStreamSynchronize(pb->st));
    return LSP_OK;
  });
}

lsp_status lsp_solve(lsp_problem* pb, int nrhs, int rhs_kind, const void* rhs, void* u, void* ws, size_t bytes,
                     lsp_rhs_info* info) {
  return guarded([&]() -> lsp_status {
    LSP_REQUIRE(pb && rhs && u, "null argument");
    LSP_REQUIRE(rhs_kind == LSP_RHS_INCIDENT || rhs_kind == LSP_RHS_G || rhs_kind == LSP_RHS_SOURCE,
                "unknown rhs kind");
    if (!pb->factored) throw Error(LSP_ERR_STATE, "lsp_factor has not succeeded on this problem");
    check_ws(pb, nrhs, true, ws, bytes);
    const Plan& P = pb->plan->p;
    const lsp_options& o = P.opts;
    const int R = o.restart;
    const long long N = P.N, NB = (long long)nrhs * N;
    hipStream_t st = pb->st;
    SolvePtrs s;
    layout_solve(P, nrhs, R, true, (void*)align_up((size_t)ws, 256), &s);
    pb->ensure_host(nrhs);
    double2* x = (double2*)u;
    LSP_HIP(hipEventRecord(pb->ev[lsp_problem::EV_SOLVE0], st));

    // g
    if (rhs_kind == LSP_RHS_INCIDENT) {
      apply_conv(pb, s, nrhs, LSP_FP64, (const double2*)rhs, s.t, false, pb->d.w2m);
      launch_scale_rhs(s.g, s.t, -1.0, NB, st);
    } else if (rhs_kind == LSP_RHS_SOURCE) {
      apply_conv(pb, s, nrhs, LSP_FP64, (const double2*)rhs, s.g, false, nullptr);  // g = K f
    } else {
      LSP_HIP(hipMemcpyAsync(s.g, rhs, NB * sizeof(double2), hipMemcpyDeviceToDevice, st));
    }
    k_fill_zero(x, NB * (long long)sizeof(double2), st);
    LSP_HIP(hipMemcpyAsync(s.r, s.g, NB * sizeof(double2), hipMemcpyDeviceToDevice, st));
    k_norm(s.r, s.partial, s.h, s.H, s.scal, -1, R, N, nrhs, nullptr, st);

    // Restarted GMRES; every stopping decision is taken on the device (same
    // rules as the host would apply) and the host only waits for the count
    // of right-hand sides still iterating.
    const GmresState gs{s.scal, s.active, s.ksz, s.iters, s.done};
    const GmresParams gp{o.tol, pb->precision == LSP_MIXED ? 1e-5 : 0.0, o.max_iters};
    const CtlView hv = lsp_problem::ctl_view(pb->ctl_dev, pb->host_cap);
    k_gmres_control(false, nrhs, gs, gp, hv, ++pb->ctl_tag, st);
    int nact = pb->wait_ctl(pb->ctl_tag);
    while (nact > 0) {
      k_cycle_init(s.H, s.gam, s.scal, R, nrhs, st);
      k_scale(s.V, s.r, s.scal, N, nrhs, s.active, st);
      int steps = 0;
      for (int k = 0; k < R; ++k) {
        double2* Vk = s.V + (size_t)k * NB;
        double2* Zk = s.Z + (size_t)k * NB;
        apply_precond(pb, s, nrhs, Vk, Zk);
        apply_conv(pb, s, nrhs, pb->precision, Zk, s.w, true, pb->d.w2m);
        k_arnoldi_orth(s.V, s.w, s.partial, s.partial2, s.h, s.H, s.scal, s.V + (size_t)(k + 1) * NB, k, R, N, nrhs,
                       s.active, st);
        k_givens(s.H, s.cs, s.sn, s.gam, k, R, nrhs, gs, gp, hv, ++pb->ctl_tag, st);
        steps = k + 1;
        if (pb->wait_ctl(pb->ctl_tag) == 0) break;
      }
      k_backsolve_update(s.H, s.gam, s.y, s.ksz, x, s.Z, R, steps, N, nrhs, st);
      // true residual in complex128
      apply_conv(pb, s, nrhs, LSP_FP64, x, s.t, true, pb->d.w2m);
      k_sub(s.r, s.g, s.t, NB, st);
      k_norm(s.r, s.partial, s.h, s.H, s.scal, -1, R, N, nrhs, nullptr, st);
      k_gmres_control(true, nrhs, gs, gp, hv, ++pb->ctl_tag, st);
      nact = pb->wait_ctl(pb->ctl_tag);
    }
    // every launch of the solve has completed (the last report is in)
    LSP_HIP(hipEventRecord(pb->ev[lsp_problem::EV_SOLVE1], st));
    LSP_HIP(hipEventSynchronize(pb->ev[lsp_problem::EV_SOLVE1]));
    const double t_setup = pb->phase_ms(lsp_problem::EV_SETUP0, lsp_problem::EV_SETUP1, true);
    const double t_factor = pb->phase_ms(lsp_problem::EV_FACTOR0, lsp_problem::EV_FACTOR1, pb->factor_timed);
    const double t_solve = pb->phase_ms(lsp_problem::EV_SOLVE0, lsp_problem::EV_SOLVE1, true);
    const CtlView hh = lsp_problem::ctl_view(pb->ctl_host, pb->host_cap);
    bool all = true;
    for (int r = 0; r < nrhs; ++r) {
      const double gnorm = hh.gnorm[r], beta = hh.beta[r];
      bool conv = gnorm == 0.0 || beta <= o.tol * gnorm;
      all = all && conv;
      if (info) {
        info[r].iters = hh.iters[r];
        info[r].converged = conv ? 1 : 0;
        info[r].relres_true = gnorm > 0 ? beta / gnorm : 0.0;
        info[r].relres_est = gnorm > 0 ? hh.est[r] / gnorm : 0.0;
        info[r].t_setup = t_setup;
        info[r].t_factor = t_factor;
        info[r].t_solve = t_solve;
      }
    }
    if (!all) throw Error(LSP_ERR_NOCONV, "GMRES reached max_iters before the tolerance");
    return LSP_OK;
  });
}

}  // extern "C"
