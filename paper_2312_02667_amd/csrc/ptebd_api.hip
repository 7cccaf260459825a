// Host runtime and C ABI of libptebd (see include/ptebd.h).
//
// The handle owns a device arena with fixed per-site slots (2 chi_cap^2 complex numbers per
// Gamma, chi_cap doubles per Lambda), a grow-only layer workspace (work matrices, rotation
// matrices, descriptors, per-gate outputs) and pinned host staging.  Bond dimensions are
// mirrored on the host; each layer reads the new dimensions back when it completes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "ptebd.h"
#include "ptebd_internal.h"

using ptebd::cplx;
using ptebd::GateDesc;
using ptebd::LayerOut;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define PT_HIP(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(PTEBD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define PT_CHECK(expr)      \
  do {                      \
    int st_ = (expr);       \
    if (st_ < 0) return st_; \
  } while (0)

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t need) {
    if (need <= bytes) return PTEBD_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    size_t alloc = std::max<size_t>(need, 256);
    if (hipMalloc(&p, alloc) != hipSuccess) {
      p = nullptr;
      return fail(PTEBD_ENOMEM, "device allocation of " + std::to_string(alloc) + " bytes failed");
    }
    bytes = alloc;
    return PTEBD_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

// Grow-only pinned host buffer.
struct HostBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t need) {
    if (need <= bytes) return PTEBD_OK;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    size_t alloc = std::max<size_t>(need, 256);
    if (hipHostMalloc(&p, alloc, hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      return fail(PTEBD_ENOMEM, "pinned host allocation failed");
    }
    bytes = alloc;
    return PTEBD_OK;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
};

struct StateInfo {
  int n = 0;
  int cap = 0;
  std::vector<int32_t> dims;  // chi_0..chi_N
  size_t gamma_off = 0;       // complex elements
  size_t lam_off = 0;         // doubles
  double prod_nu = 1.0;
  double prod_fid = 1.0;
};

// One bond update: gate (host pointer to 32 doubles) at q of state s, or the identity; chi
// is its truncation bound (0: a tSU step, bounded by chi_{q+1} only).
struct Item {
  int s;
  int q;
  const double* gate;
  int chi;
};

struct UpdateResult {
  std::vector<int32_t> k, r, sweeps;
  std::vector<double> eps, nu;
  int max_sweeps = 0;
  int n_unconverged = 0;
};

// Event-based per-kernel timing (enabled by ptebd_set_profiling).
struct Prof {
  bool on = false;
  struct Pend {
    int kind;
    hipEvent_t a, b;
    int count;  // launches the interval stands for (-1: a sweep queued past convergence,
                // whose early-exit launches are not counted)
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pend> pending;
  ptebd_kernel_stats st[PTEBD_KERNEL_COUNT];
  Prof() { reset(); }
  void reset() {
    for (auto& x : st) x = ptebd_kernel_stats{0.0, 0, 0.0, 0.0};
  }
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  // Intervals of one kernel class running on two streams at once, on a common clock (events
  // relative to `ref`): per class, their union is the time that class occupied the GPU, and
  // `count` the launches over all gates the interval stands for (half a launch per half of
  // the gates).
  struct Span {
    int kind;
    hipEvent_t a, b;
    double count;
  };
  hipEvent_t ref = nullptr;
  std::vector<Span> spans;
  void harvest_spans() {
    for (int kind = 0; kind < PTEBD_KERNEL_COUNT; ++kind) {
      std::vector<std::pair<float, float>> iv;
      double count = 0.0;
      for (const Span& sp : spans) {
        if (sp.kind != kind || sp.count < 0) continue;
        float a = 0.f, b = 0.f;
        if (ref && hipEventElapsedTime(&a, ref, sp.a) == hipSuccess &&
            hipEventElapsedTime(&b, ref, sp.b) == hipSuccess)
          iv.push_back({a, b});
        count += sp.count;
      }
      if (iv.empty()) continue;
      std::sort(iv.begin(), iv.end());
      double total = 0.0, lo = 0.0, hi = -1.0;
      for (const auto& x : iv) {
        if (x.first > hi) {
          if (hi > lo) total += hi - lo;
          lo = x.first;
          hi = x.second;
        } else if (x.second > hi) {
          hi = x.second;
        }
      }
      if (hi > lo) total += hi - lo;
      st[kind].total_ms += total;
      st[kind].launches += (int64_t)std::llround(count);
    }
    for (const Span& sp : spans) {
      pool.push_back(sp.a);
      pool.push_back(sp.b);
    }
    if (ref) pool.push_back(ref);
    ref = nullptr;
    spans.clear();
  }
  // Harvest finished launches (the stream has been synchronized).
  void harvest() {
    for (const Pend& p : pending) {
      float ms = 0.f;
      if (p.count >= 0 && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        st[p.kind].total_ms += ms;
        st[p.kind].launches += p.count;
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  void release() {
    harvest();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
  }
};

// Launch `fn` on `stream`, bracketed by events when profiling is on.
template <class F>
void timed(Prof* pf, int kind, hipStream_t stream, F fn) {
  if (!pf || !pf->on) {
    fn();
    return;
  }
  hipEvent_t a = pf->get(), b = pf->get();
  if (!a || !b) {
    fn();
    return;
  }
  (void)hipEventRecord(a, stream);
  fn();
  (void)hipEventRecord(b, stream);
  pf->pending.push_back({kind, a, b, 1});
}

// Launch `fn` on one of two concurrent streams, its interval recorded for the union of its
// class (standing for `count` launches over all gates) when profiling is on.
template <class F>
int timed_span(Prof* pf, int kind, hipStream_t stream, double count, F fn) {
  hipEvent_t a = pf && pf->on && pf->ref ? pf->get() : nullptr;
  hipEvent_t b = a ? pf->get() : nullptr;
  if (a && b && hipEventRecord(a, stream) != hipSuccess) return PTEBD_EDEVICE;
  fn();
  if (a && b) {
    if (hipEventRecord(b, stream) != hipSuccess) return PTEBD_EDEVICE;
    pf->spans.push_back({kind, a, b, count});
  } else {
    if (a) pf->pool.push_back(a);
    if (b) pf->pool.push_back(b);
  }
  return PTEBD_OK;
}

// Instantiated graphs of one Jacobi sweep (its rounds and the convergence check), keyed by
// every argument the captured launches carry; captured on a private stream and launched on
// the pipeline's stream.  A few entries suffice (a layer's shapes repeat); the least recently
// used one is replaced.
struct SweepGraphs {
  struct Entry {
    std::string key;
    hipGraphExec_t exec;
    uint64_t used;
  };
  std::vector<Entry> entries;
  hipStream_t capture = nullptr;
  uint64_t tick = 0;
  static constexpr size_t kMax = 12;
  void release() {
    for (Entry& e : entries) (void)hipGraphExecDestroy(e.exec);
    entries.clear();
    if (capture) (void)hipStreamDestroy(capture);
    capture = nullptr;
  }
};

double unit_roundoff(int precision) {
  return precision == PTEBD_FP64 ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
}

}  // namespace

struct ptebd_mps {
  int device = 0;
  hipStream_t stream = nullptr;
  int precision = PTEBD_FP64;
  size_t celem = 16;  // bytes per complex element
  std::vector<StateInfo> st;
  DevBuf gamma, lam;
  DevBuf work, desc, gates, outbuf, qscratch, renv, qout, aux, samp;
  HostBuf h_desc, h_gates, h_out, h_small;
  Prof prof;
  int max_sweeps = 30;
  double tol_factor = 4.0;
  int inner_sweeps = 1;
  double inner_repeat = 0.0;
  int sort_pairs = 1;
  int precondition = 1;  // FP32 handles only
  int streams = 2;       // Jacobi sweeps of a large batch on two streams
  int block_cols = 16;   // Jacobi block width (32: FP32 handles only)
  int graphs = 1;        // each Jacobi sweep as one captured HIP graph
  SweepGraphs sweep_graphs;
  hipEvent_t ev_sweep[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [pipeline][parity]
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // second stream of the Jacobi sweeps and its fork / join events, created on first use
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  char* gamma_slot(int s, int q) const {
    const StateInfo& si = st[s];
    return (char*)gamma.p + (si.gamma_off + (size_t)q * 2 * si.cap * si.cap) * celem;
  }
  double* lam_slot(int s, int i) const {
    const StateInfo& si = st[s];
    return (double*)lam.p + si.lam_off + (size_t)i * si.cap;
  }
};

namespace {

// Layout of the per-gate output block inside outbuf.
struct OutLayout {
  size_t sig, perm, k, r, eps, nu, sweeps, conv, offbits, counters, ps, gmax, work, rstart,
      counters2, total;
  int nslot, nbmax;
};

// Column-block pairs per round of the block Jacobi for matrices of up to cmax columns.
int pair_slots(int cmax) {
  const int nb = (cmax + 15) / 16;
  return std::max(2, nb + (nb & 1)) / 2;
}

OutLayout out_layout(int n, int cmax) {
  OutLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  L.sig = take(sizeof(double) * (size_t)n * cmax);
  L.perm = take(sizeof(int32_t) * (size_t)n * cmax);
  L.k = take(sizeof(int32_t) * n);
  L.r = take(sizeof(int32_t) * n);
  L.eps = take(sizeof(double) * n);
  L.nu = take(sizeof(double) * n);
  L.sweeps = take(sizeof(int32_t) * n);
  L.conv = take(sizeof(int32_t) * n);
  L.offbits = take(sizeof(uint32_t) * n);
  L.counters = take(sizeof(int32_t) * 4);
  L.ps = take(sizeof(int32_t) * (size_t)n * cmax);
  L.gmax = take(sizeof(double) * n);
  L.nslot = pair_slots(cmax);
  L.work = take(sizeof(uint32_t) * 2 * (size_t)n * L.nslot);
  L.nbmax = (cmax + 15) / 16;
  L.rstart = take(sizeof(int32_t) * (size_t)n * L.nbmax);
  L.counters2 = take(sizeof(int32_t) * 4);  // the second half's sweep counters
  L.total = off;
  return L;
}

LayerOut make_layer_out(void* base, const OutLayout& L, int cmax) {
  char* b = (char*)base;
  LayerOut o{};
  o.sig = (double*)(b + L.sig);
  o.perm = (int32_t*)(b + L.perm);
  o.k = (int32_t*)(b + L.k);
  o.r = (int32_t*)(b + L.r);
  o.eps = (double*)(b + L.eps);
  o.nu = (double*)(b + L.nu);
  o.sweeps = (int32_t*)(b + L.sweeps);
  o.conv = (int32_t*)(b + L.conv);
  o.offbits = (uint32_t*)(b + L.offbits);
  o.counters = (int32_t*)(b + L.counters);
  o.work = (uint32_t*)(b + L.work);
  o.nslot = L.nslot;
  o.rstart = (int32_t*)(b + L.rstart);
  o.nbmax = L.nbmax;
  o.triangular = 0;
  o.block_cols = 16;
  o.cmax = cmax;
  return o;
}

// The per-gate outputs of gates off.. of a layer (their own sweep counters).
LayerOut shift_out(const LayerOut& o, int off, int32_t* counters) {
  LayerOut r = o;
  r.sig += (size_t)off * o.cmax;
  r.perm += (size_t)off * o.cmax;
  r.k += off;
  r.r += off;
  r.eps += off;
  r.nu += off;
  r.sweeps += off;
  r.conv += off;
  r.offbits += off;
  r.counters = counters;
  r.work += (size_t)off * 2 * o.nslot;
  r.rstart += (size_t)off * o.nbmax;
  return r;
}

// A second stream: one half of a large batch runs its whole pipeline on it.
struct SplitStreams {
  hipStream_t s2;
  hipEvent_t ev_fork, ev_join;
  int32_t* counters2;  // device, 4 ints
};

// One round of the block Jacobi with the block width of lo (32-column blocks: FP32 only).
template <class T>
void launch_round(const GateDesc* d_desc, int n, int round, int nbp, const LayerOut& lo,
                  double tol_scale, int inner_sweeps, double inner_repeat, int sort_pairs,
                  int prev_slot, hipStream_t stream) {
  if (sizeof(T) == 4 && lo.block_cols == 32)
    ptebd::launch_jacobi_round64(d_desc, n, round, nbp, lo, tol_scale, inner_sweeps,
                                 inner_repeat, sort_pairs, prev_slot, stream);
  else
    ptebd::launch_jacobi_round<T>(d_desc, n, round, nbp, lo, tol_scale, inner_sweeps,
                                  inner_repeat, sort_pairs, prev_slot, stream);
}

// Players of one sweep's tournament: the block count of max_c columns, made even.
int tournament_players(int max_c, int block_cols) {
  const int nb = (max_c + block_cols - 1) / block_cols;
  return std::max(2, nb + (nb & 1));
}

// What one pipeline's sweeps need: its gates, their outputs and the SVD controls.
struct SweepArgs {
  const GateDesc* d;
  int n, nbp;
  LayerOut lo;
  double tol_factor, u;
  int inner_sweeps;
  double inner_repeat;
  int sort_pairs;
};

template <class X>
void append_key(std::string& k, const X& x) {
  static_assert(std::is_arithmetic<X>::value || std::is_pointer<X>::value,
                "keys are built from scalar fields (a struct's padding bytes are indeterminate)");
  k.append(reinterpret_cast<const char*>(&x), sizeof(X));
}

// The fields of a LayerOut a sweep's launches read, one by one.
void append_key(std::string& k, const LayerOut& o) {
  for (const void* p : {(const void*)o.sig, (const void*)o.perm, (const void*)o.k,
                        (const void*)o.r, (const void*)o.eps, (const void*)o.nu,
                        (const void*)o.sweeps, (const void*)o.conv, (const void*)o.offbits,
                        (const void*)o.counters, (const void*)o.work, (const void*)o.rstart})
    append_key(k, p);
  for (int32_t v : {o.nslot, o.nbmax, o.triangular, o.block_cols, o.cmax})
    append_key(k, v);
}

// Sweep s of a pipeline on `stream`: its nbp - 1 rounds and the convergence check that counts
// the unconverged gates into lo.counters[s & 1].  Every round of a sweep s > 0 returns at once
// when the previous sweep's count is zero, so a sweep queued before the host has read that
// count costs only its empty launches.  With a graph cache (sg), the sweep is one launch of a
// captured graph; the sweeps s > 0 of one parity share a graph.
template <class T>
int launch_sweep(SweepGraphs* sg, hipStream_t stream, const SweepArgs& a, int s) {
  const int prev_slot = s == 0 ? -1 : ((s - 1) & 1);
  auto body = [&](hipStream_t st) {
    for (int r = 0; r < a.nbp - 1; ++r)
      launch_round<T>(a.d, a.n, r, a.nbp, a.lo, a.tol_factor * a.u, a.inner_sweeps,
                      a.inner_repeat, a.sort_pairs, prev_slot, st);
    ptebd::launch_sweep_check(a.d, a.n, s & 1, a.tol_factor, a.u, a.lo, st);
  };
  if (!sg) {
    body(stream);
    PT_HIP(hipGetLastError());
    return PTEBD_OK;
  }
  std::string key;
  const int variant = s == 0 ? 0 : 1 + (s & 1);
  append_key(key, (int)sizeof(T));
  append_key(key, a.d);
  append_key(key, a.n);
  append_key(key, a.nbp);
  append_key(key, a.lo);
  append_key(key, a.tol_factor);
  append_key(key, a.u);
  append_key(key, a.inner_sweeps);
  append_key(key, a.inner_repeat);
  append_key(key, a.sort_pairs);
  append_key(key, variant);
  SweepGraphs::Entry* hit = nullptr;
  for (auto& e : sg->entries)
    if (e.key == key) hit = &e;
  if (!hit) {
    if (!sg->capture)
      PT_HIP(hipStreamCreateWithFlags(&sg->capture, hipStreamNonBlocking));
    PT_HIP(hipStreamBeginCapture(sg->capture, hipStreamCaptureModeThreadLocal));
    body(sg->capture);
    hipGraph_t graph = nullptr;
    const hipError_t launched = hipGetLastError();
    const hipError_t ended = hipStreamEndCapture(sg->capture, &graph);
    if (launched != hipSuccess || ended != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(PTEBD_EDEVICE, "capture of a Jacobi sweep graph failed");
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t inst = hipGraphInstantiateWithFlags(&exec, graph, 0);
    (void)hipGraphDestroy(graph);
    if (inst != hipSuccess || !exec)
      return fail(PTEBD_EDEVICE, "instantiation of a Jacobi sweep graph failed");
    if (sg->entries.size() >= SweepGraphs::kMax) {
      auto lru = std::min_element(sg->entries.begin(), sg->entries.end(),
                                  [](const SweepGraphs::Entry& x, const SweepGraphs::Entry& y) {
                                    return x.used < y.used;
                                  });
      (void)hipGraphExecDestroy(lru->exec);
      sg->entries.erase(lru);
    }
    sg->entries.push_back({key, exec, 0});
    hit = &sg->entries.back();
  }
  hit->used = ++sg->tick;
  PT_HIP(hipGraphLaunch(hit->exec, stream));
  return PTEBD_OK;
}

// A pipeline's sweeps driven from the device side: sweep s + 1 is queued before the host
// reads sweep s's count of unconverged gates (one 4-byte copy and an event per sweep), so
// the device never waits for the host between sweeps; a sweep queued past convergence
// returns at once and is not counted in the profile.
template <class T>
struct SweepDriver {
  SweepGraphs* sg;
  hipStream_t stream;
  SweepArgs a;
  int max_sweeps;
  int32_t* h_cnt;      // two pinned host ints (sweep parity)
  hipEvent_t ev[2];    // recorded after each sweep's count copy
  Prof* pf;
  double span_count;   // > 0: profile as a span (two concurrent pipelines), else per sweep
  int issued = 0;      // sweeps queued
  int checked = -1;    // last sweep whose count was read
  long prof_idx[64];   // profile entry of each queued sweep (by sweep index mod 64)

  int issue(int s) {
    prof_idx[s & 63] = -1;
    const bool prof = pf && pf->on;
    if (prof && span_count > 0.0) {
      prof_idx[s & 63] = pf->ref ? (long)pf->spans.size() : -1;
      int st_ = PTEBD_OK;
      PT_CHECK(timed_span(pf, PTEBD_KERNEL_JACOBI, stream, span_count,
                          [&] { st_ = launch_sweep<T>(sg, stream, a, s); }));
      PT_CHECK(st_);
    } else if (prof) {
      prof_idx[s & 63] = (long)pf->pending.size();
      int st_ = PTEBD_OK;
      timed(pf, PTEBD_KERNEL_JACOBI, stream, [&] { st_ = launch_sweep<T>(sg, stream, a, s); });
      PT_CHECK(st_);
      if ((size_t)prof_idx[s & 63] < pf->pending.size())
        pf->pending[prof_idx[s & 63]].count = a.nbp - 1;
      else
        prof_idx[s & 63] = -1;
    } else {
      PT_CHECK(launch_sweep<T>(sg, stream, a, s));
    }
    PT_HIP(hipMemcpyAsync(h_cnt + (s & 1), a.lo.counters + (s & 1), sizeof(int32_t),
                          hipMemcpyDeviceToHost, stream));
    PT_HIP(hipEventRecord(ev[s & 1], stream));
    issued = s + 1;
    return PTEBD_OK;
  }
  // queue the first sweeps
  int start() {
    PT_CHECK(issue(0));
    if (max_sweeps > 1) PT_CHECK(issue(1));
    return PTEBD_OK;
  }
  // wait for the next unread sweep; *done = 1 with *rem the final count when the pipeline
  // has converged or used its sweeps, else the following sweep is queued
  int step(int* done, int* rem) {
    const int s = checked + 1;
    PT_HIP(hipEventSynchronize(ev[s & 1]));
    checked = s;
    *rem = h_cnt[s & 1];
    if (*rem == 0 || s + 1 >= max_sweeps) {
      *done = 1;
      // a sweep queued after this one found the batch converged and did nothing
      for (int t = s + 1; t < issued; ++t) {
        const long idx = prof_idx[t & 63];
        if (idx < 0 || !pf) continue;
        if (span_count > 0.0) {
          if ((size_t)idx < pf->spans.size()) pf->spans[idx].count = -1.0;
        } else if ((size_t)idx < pf->pending.size()) {
          pf->pending[idx].count = -1;
        }
      }
      return PTEBD_OK;
    }
    *done = 0;
    if (s + 2 < max_sweeps && issued <= s + 2) PT_CHECK(issue(s + 2));
    return PTEBD_OK;
  }
};

int sweep_events(ptebd_mps* h, int k, hipEvent_t ev[2]) {
  for (int j = 0; j < 2; ++j) {
    if (!h->ev_sweep[k][j])
      PT_HIP(hipEventCreateWithFlags(&h->ev_sweep[k][j], hipEventDisableTiming));
    ev[j] = h->ev_sweep[k][j];
  }
  return PTEBD_OK;
}

// Sweeps of the block Jacobi SVD on descriptors already on the device, on one stream.  With
// a handle: the device-driven sweeps of SweepDriver (graphs when the handle enables them);
// without one (the stand-alone batched SVD entry points): one sweep at a time, each followed
// by a read of its count.
template <class T>
int run_jacobi(ptebd_mps* h, hipStream_t stream, const GateDesc* d_desc, int n, int max_c,
               const LayerOut& lo, int precision, int max_sweeps, double tol_factor,
               int inner_sweeps, double inner_repeat, int sort_pairs, int32_t* h_counter,
               int* n_unconverged, Prof* pf) {
  ptebd::launch_jacobi_init<T>(d_desc, n, max_c, lo, stream);
  const SweepArgs a{d_desc, n, tournament_players(max_c, lo.block_cols), lo, tol_factor,
                    unit_roundoff(precision), inner_sweeps, inner_repeat, sort_pairs};
  if (!h) {
    int remaining = n;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
      PT_CHECK(launch_sweep<T>(nullptr, stream, a, sweep));
      PT_HIP(hipMemcpyAsync(h_counter, lo.counters + (sweep & 1), sizeof(int32_t),
                            hipMemcpyDeviceToHost, stream));
      PT_HIP(hipStreamSynchronize(stream));
      remaining = *h_counter;
      if (remaining == 0) break;
    }
    *n_unconverged = remaining;
    return PTEBD_OK;
  }
  SweepDriver<T> drv{h->graphs ? &h->sweep_graphs : nullptr, stream, a, max_sweeps, h_counter,
                     {nullptr, nullptr}, pf, 0.0};
  PT_CHECK(sweep_events(h, 0, drv.ev));
  PT_CHECK(drv.start());
  int done = 0, rem = n;
  while (!done) PT_CHECK(drv.step(&done, &rem));
  if (pf) {
    PT_HIP(hipStreamSynchronize(stream));
    pf->harvest();
  }
  *n_unconverged = rem;
  return PTEBD_OK;
}

// The handle's split-stream resources when its batch qualifies (nullptr: one stream).
const SplitStreams* split_for(ptebd_mps* h, int n, const OutLayout& L, SplitStreams* out) {
  if (h->streams < 2 || n < 64) return nullptr;
  if (!h->stream2) {
    if (hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess)
      return nullptr;  // fall back to one stream
  }
  out->s2 = h->stream2;
  out->ev_fork = h->ev_fork;
  out->ev_join = h->ev_join;
  out->counters2 = (int32_t*)((char*)h->outbuf.p + L.counters2);
  return out;
}

// A large batch as two independent pipelines: gates [0, n/2) on `stream`, [n/2, n) on the
// second stream, each running theta, the preconditioning, its own Jacobi sweeps, finalize
// and the recovery (the write-back follows for the whole batch once its errors have been
// checked).  The host advances each half's sweeps as soon as its
// own convergence counter is read, so one half's theta and preconditioning, sweep
// boundaries and last launches overlap the other half's rounds.  Jacobi time is the union
// of the intervals in which either half's rounds ran (events on one clock), each round over
// half the gates counting as half a launch.  Both streams have drained on return.
template <class T>
int run_split(ptebd_mps* h, const SplitStreams& sp, const GateDesc* d_desc,
              const GateDesc* d_jdesc, int n, int max_c, int max_r,
              int max_tiles, bool pre, double cutoff, const LayerOut& lo,
              const ptebd::PrecondOut& po, int32_t* h_counter, int* n_unconverged) {
  hipStream_t stream = h->stream;
  Prof* pf = &h->prof;
  const bool prof = pf->on;
  const int n1 = n / 2;
  const int nn[2] = {n1, n - n1};
  const int off[2] = {0, n1};
  hipStream_t st[2] = {stream, sp.s2};
  const LayerOut oo[2] = {lo, shift_out(lo, n1, sp.counters2)};
  ptebd::PrecondOut pp[2] = {po, po};
  pp[1].ps += (size_t)n1 * po.cmax;
  pp[1].gmax += n1;
  const int nbp = tournament_players(max_c, lo.block_cols);
  const double u = unit_roundoff(h->precision);
  if (prof) {
    pf->ref = pf->get();
    if (pf->ref) PT_HIP(hipEventRecord(pf->ref, stream));
  }
  // the second stream starts after everything already queued on the first
  PT_HIP(hipEventRecord(sp.ev_fork, stream));
  PT_HIP(hipStreamWaitEvent(sp.s2, sp.ev_fork, 0));
  // whatever way this returns, neither stream is left running on the batch's buffers
  struct Drain {
    hipStream_t a, b;
    ~Drain() {
      (void)hipStreamSynchronize(a);
      (void)hipStreamSynchronize(b);
    }
  } drain{stream, sp.s2};
  auto front = [&](int k) {
    const GateDesc* dd = d_desc + off[k];
    PT_CHECK(timed_span(pf, PTEBD_KERNEL_THETA, st[k], 0.5,
                        [&] { ptebd::launch_theta<T>(dd, nn[k], max_tiles, st[k]); }));
    if (pre)
      PT_CHECK(timed_span(pf, PTEBD_KERNEL_PRECOND, st[k], 0.5, [&] {
        ptebd::launch_colsort(dd, nn[k], pp[k], st[k]);
        ptebd::launch_gram64(dd, nn[k], max_c, pp[k], st[k]);
        ptebd::launch_cholesky(dd, nn[k], max_c, pp[k], st[k]);
        ptebd::launch_xinit(d_jdesc + off[k], nn[k], max_c, st[k]);
      }));
    ptebd::launch_jacobi_init<T>(d_jdesc + off[k], nn[k], max_c, oo[k], st[k]);
    return PTEBD_OK;
  };
  auto back = [&](int k) {
    const GateDesc* jd = d_jdesc + off[k];
    PT_CHECK(timed_span(pf, PTEBD_KERNEL_FINALIZE, st[k], 0.5,
                        [&] { ptebd::launch_finalize<T>(jd, nn[k], cutoff, oo[k], st[k]); }));
    if (pre)
      PT_CHECK(timed_span(pf, PTEBD_KERNEL_PRECOND, st[k], 0.0, [&] {
        ptebd::launch_recover(d_desc + off[k], jd, nn[k], max_r, max_c, pp[k], oo[k], st[k]);
      }));
    return PTEBD_OK;
  };
  // each half's sweeps run device-driven (SweepDriver); the host serves whichever half's
  // next count is due, queueing that half's next sweep or its finalize and recovery
  SweepDriver<T> drv[2] = {
      {h->graphs ? &h->sweep_graphs : nullptr, st[0],
       SweepArgs{d_jdesc, nn[0], nbp, oo[0], h->tol_factor, u, h->inner_sweeps,
                 h->inner_repeat, h->sort_pairs},
       h->max_sweeps, h_counter, {nullptr, nullptr}, pf, 0.5 * (nbp - 1)},
      {h->graphs ? &h->sweep_graphs : nullptr, st[1],
       SweepArgs{d_jdesc + off[1], nn[1], nbp, oo[1], h->tol_factor, u, h->inner_sweeps,
                 h->inner_repeat, h->sort_pairs},
       h->max_sweeps, h_counter + 2, {nullptr, nullptr}, pf, 0.5 * (nbp - 1)}};
  bool active[2] = {true, true};
  for (int k = 0; k < 2; ++k) {
    PT_CHECK(sweep_events(h, k, drv[k].ev));
    PT_CHECK(front(k));
    PT_CHECK(drv[k].start());
  }
  PT_HIP(hipGetLastError());
  int unconv = 0;
  while (active[0] || active[1]) {
    for (int k = 0; k < 2; ++k) {
      if (!active[k]) continue;
      int done = 0, rem = 0;
      PT_CHECK(drv[k].step(&done, &rem));
      if (done) {
        active[k] = false;
        unconv += rem;
        PT_CHECK(back(k));
      }
      PT_HIP(hipGetLastError());
    }
  }
  for (int k = 0; k < 2; ++k) PT_HIP(hipStreamSynchronize(st[k]));
  if (prof) {
    pf->harvest();
    pf->harvest_spans();
  }
  *n_unconverged = unconv;
  return PTEBD_OK;
}

// One batch of independent bond updates (all gates of a layer, or one PtSU half-step).
template <class T>
int run_updates(ptebd_mps* h, const std::vector<Item>& items, double cutoff,
                int stabilize, int eps_mode, UpdateResult* res) {
  const int n = (int)items.size();
  res->k.assign(n, 0);
  res->r.assign(n, 0);
  res->sweeps.assign(n, 0);
  res->eps.assign(n, 0.0);
  res->nu.assign(n, 1.0);
  res->max_sweeps = 0;
  res->n_unconverged = 0;
  if (n == 0) return PTEBD_OK;
  if (n > 65535) return fail(PTEBD_EINVAL, "too many bond updates in one batch (max 65535)");

  // The FP32 path preconditions the SVD (column sort, FP64 Gram, Cholesky, Jacobi on R^H);
  // its per-gate workspace adds the Gram matrix (C x C complex FP64) and U S (R x C).
  const bool pre = sizeof(T) == 4 && h->precondition;
  std::vector<size_t> woff(n), voff(n), goff(n), loff(n);
  size_t total = 0;
  int max_c = 1, max_r = 1, max_tiles = 1, cmax = 1;
  std::vector<GateDesc> descs(n);
  for (int i = 0; i < n; ++i) {
    const StateInfo& si = h->st[items[i].s];
    const int q = items[i].q;
    GateDesc& d = descs[i];
    std::memset(&d, 0, sizeof(d));
    d.cl = si.dims[q];
    d.cm = si.dims[q + 1];
    d.cr = si.dims[q + 2];
    const int m = 2 * d.cl, nn = 2 * d.cr;
    d.transposed = nn > m ? 1 : 0;
    d.R = std::max(m, nn);
    d.C = std::min(m, nn);
    d.has_gate = items[i].gate != nullptr ? 1 : 0;
    // tSU (item chi 0): theta = A B has rank <= chi_{q+1}, so the kept dimension is
    // bounded by it; singular values beyond it are rounding noise of the precision.
    d.chi_max = items[i].chi > 0 ? items[i].chi : d.cm;
    d.stabilize = stabilize;
    d.eps_mode = eps_mode;
    woff[i] = total;
    total += (size_t)d.R * d.C;
    voff[i] = total;
    total += (size_t)d.C * d.C;
    if (pre) {
      total += total & 1;  // the complex FP64 Gram matrix is 16-byte aligned
      goff[i] = total;
      total += 2 * (size_t)d.C * d.C;
      loff[i] = total;
      total += (size_t)d.R * d.C;
    }
    max_c = std::max(max_c, d.C);
    max_r = std::max(max_r, d.R);
    cmax = std::max(cmax, d.C);
    max_tiles = std::max(max_tiles, ((d.cl + 31) / 32) * ((d.cr + 31) / 32));
  }
  const OutLayout L = out_layout(n, cmax);
  PT_CHECK(h->work.ensure(total * sizeof(cplx<T>)));
  const int ndesc = pre ? 3 * n : n;  // theta, Jacobi and write-back descriptors
  PT_CHECK(h->desc.ensure(sizeof(GateDesc) * ndesc));
  PT_CHECK(h->gates.ensure(sizeof(double) * 32 * n));
  PT_CHECK(h->outbuf.ensure(L.total));
  PT_CHECK(h->h_desc.ensure(sizeof(GateDesc) * ndesc));
  PT_CHECK(h->h_gates.ensure(sizeof(double) * 32 * n));
  PT_CHECK(h->h_out.ensure(L.total));
  PT_CHECK(h->h_small.ensure(64));

  char* wbase = (char*)h->work.p;
  double* hg = (double*)h->h_gates.p;
  for (int i = 0; i < n; ++i) {
    GateDesc& d = descs[i];
    const int s = items[i].s, q = items[i].q;
    d.gq = h->gamma_slot(s, q);
    d.gq1 = h->gamma_slot(s, q + 1);
    d.lam_l = h->lam_slot(s, q);
    d.lam_m = h->lam_slot(s, q + 1);
    d.lam_r = h->lam_slot(s, q + 2);
    d.w = wbase + woff[i] * sizeof(cplx<T>);
    d.v = wbase + voff[i] * sizeof(cplx<T>);
    d.gram = pre ? wbase + goff[i] * sizeof(cplx<T>) : nullptr;
    d.left = pre ? wbase + loff[i] * sizeof(cplx<T>) : nullptr;
    if (items[i].gate) {
      std::memcpy(hg + 32 * i, items[i].gate, 32 * sizeof(double));
      d.gate = (const double*)h->gates.p + 32 * i;
    } else {
      d.gate = nullptr;
    }
  }
  std::memcpy(h->h_desc.p, descs.data(), sizeof(GateDesc) * n);
  if (pre) {
    // Jacobi on X = R^H (C x C, in the V slot, no right vectors kept); write-back from
    // U S (left) and the right vectors (stored in the Gram buffer)
    GateDesc* jd = (GateDesc*)h->h_desc.p + n;
    GateDesc* wd = (GateDesc*)h->h_desc.p + 2 * n;
    for (int i = 0; i < n; ++i) {
      jd[i] = descs[i];
      jd[i].w = descs[i].v;
      jd[i].v = nullptr;
      jd[i].R = descs[i].C;
      wd[i] = descs[i];
      wd[i].w = descs[i].left;
      wd[i].v = descs[i].gram;
    }
  }
  hipStream_t stream = h->stream;
  PT_HIP(hipMemcpyAsync(h->desc.p, h->h_desc.p, sizeof(GateDesc) * ndesc, hipMemcpyHostToDevice,
                        stream));
  PT_HIP(hipMemcpyAsync(h->gates.p, h->h_gates.p, sizeof(double) * 32 * n, hipMemcpyHostToDevice,
                        stream));
  const GateDesc* d_desc = (const GateDesc*)h->desc.p;
  const GateDesc* d_jdesc = pre ? d_desc + n : d_desc;
  const GateDesc* d_wdesc = pre ? d_desc + 2 * n : d_desc;
  LayerOut lo = make_layer_out(h->outbuf.p, L, cmax);
  lo.triangular = pre ? 1 : 0;  // the Jacobi then starts from X = R^H, lower triangular
  lo.block_cols = sizeof(T) == 4 ? h->block_cols : 16;
  ptebd::PrecondOut po;
  po.ps = (int32_t*)((char*)h->outbuf.p + L.ps);
  po.gmax = (double*)((char*)h->outbuf.p + L.gmax);
  po.cmax = cmax;

  Prof* pf = &h->prof;
  int n_unconv = 0;
  SplitStreams sp;
  const SplitStreams* split = split_for(h, n, L, &sp);
  if (split) {
    PT_CHECK(run_split<T>(h, *split, d_desc, d_jdesc, n, max_c, max_r, max_tiles, pre,
                          cutoff, lo, po, (int32_t*)h->h_small.p, &n_unconv));
  } else {
    timed(pf, PTEBD_KERNEL_THETA, stream, [&] { ptebd::launch_theta<T>(d_desc, n, max_tiles, stream); });
    PT_HIP(hipGetLastError());
    if (pre)
      timed(pf, PTEBD_KERNEL_PRECOND, stream, [&] {
        ptebd::launch_colsort(d_desc, n, po, stream);
        ptebd::launch_gram64(d_desc, n, max_c, po, stream);
        ptebd::launch_cholesky(d_desc, n, max_c, po, stream);
        ptebd::launch_xinit(d_jdesc, n, max_c, stream);
      });
    PT_HIP(hipGetLastError());
    PT_CHECK(run_jacobi<T>(h, stream, d_jdesc, n, max_c, lo, h->precision, h->max_sweeps,
                           h->tol_factor, h->inner_sweeps, h->inner_repeat, h->sort_pairs,
                           (int32_t*)h->h_small.p, &n_unconv, pf));
    timed(pf, PTEBD_KERNEL_FINALIZE, stream, [&] { ptebd::launch_finalize<T>(d_jdesc, n, cutoff, lo, stream); });
    if (pre)
      timed(pf, PTEBD_KERNEL_PRECOND, stream, [&] {
        ptebd::launch_recover(d_desc, d_jdesc, n, max_r, max_c, po, lo, stream);
      });
    PT_HIP(hipGetLastError());
  }
  // copy back the small per-gate outputs (k .. counters are contiguous after perm)
  PT_HIP(hipMemcpyAsync((char*)h->h_out.p + L.k, (char*)h->outbuf.p + L.k, L.ps - L.k,
                        hipMemcpyDeviceToHost, stream));
  PT_HIP(hipStreamSynchronize(stream));
  const char* ho = (const char*)h->h_out.p;
  const int32_t* hk = (const int32_t*)(ho + L.k);
  const int32_t* hr = (const int32_t*)(ho + L.r);
  const double* he = (const double*)(ho + L.eps);
  const double* hn = (const double*)(ho + L.nu);
  const int32_t* hs = (const int32_t*)(ho + L.sweeps);
  int32_t hc[4];
  std::memcpy(hc, ho + L.counters, sizeof(hc));
  if (split) {  // the second half's finalize flags its errors in its own counters
    int32_t c2[4];
    PT_HIP(hipMemcpy(c2, (char*)h->outbuf.p + L.counters2, sizeof(c2), hipMemcpyDeviceToHost));
    hc[2] |= c2[2];
  }
  // Nothing of the state has been written so far: a batch with an error returns here and
  // leaves Gamma, Lambda and the bond dimensions as they were.
  if (hc[2] & 1) return fail(PTEBD_EANNIHILATED, "a two-site wavefunction vanished or eps >= 1");
  if (hc[2] & 2) return fail(PTEBD_ENONFINITE, "non-finite singular value, eps or nu produced");
  // Algorithm 1 compresses a state's layer (nu, then PtSU) only when some of its gates had
  // r > chi; the write-back sets Lambda[q+1] = nu sigma[:k] for the gates of such states and
  // sigma[:k] for the others.
  std::vector<char> trig(h->st.size(), 0);
  if (stabilize)
    for (int i = 0; i < n; ++i)
      if (items[i].chi > 0 && hr[i] > items[i].chi) trig[items[i].s] = 1;
  int32_t* happ = (int32_t*)h->h_gates.p;  // the gates' staging is free again
  for (int i = 0; i < n; ++i) happ[i] = trig[items[i].s] ? 1 : 0;
  if (stabilize)
    PT_HIP(hipMemcpyAsync(h->gates.p, happ, sizeof(int32_t) * n, hipMemcpyHostToDevice, stream));
  const int32_t* d_apply = stabilize ? (const int32_t*)h->gates.p : nullptr;
  timed(pf, PTEBD_KERNEL_WRITEBACK, stream,
        [&] { ptebd::launch_writeback<T>(d_wdesc, n, d_apply, lo, stream); });
  PT_HIP(hipGetLastError());
  PT_HIP(hipStreamSynchronize(stream));
  for (int i = 0; i < n; ++i) {
    res->k[i] = hk[i];
    res->r[i] = hr[i];
    res->eps[i] = he[i];
    res->nu[i] = (stabilize && happ[i]) ? hn[i] : 1.0;
    res->sweeps[i] = hs[i];
    res->max_sweeps = std::max(res->max_sweeps, hs[i]);
    h->st[items[i].s].dims[items[i].q + 1] = hk[i];
  }
  res->n_unconverged = n_unconv;
  if (pf->on) {
    pf->harvest();
    const double ce = (double)sizeof(cplx<T>);
    // executed Jacobi rows: with b-column blocks a pair's Gram matrix over r rows forms the
    // upper 16 x 16 complex tiles of its 2b x 2b matrix, 3 (b = 16) or 10 (b = 32) tiles of
    // 2048 r flops each, reading 2b r complex entries; a rotation of r rows (W's, plus V's)
    // costs 8 (2b)^2 r flops and reads and writes 2b r complex entries each way
    const size_t wn = sizeof(uint32_t) * 2 * (size_t)n * L.nslot;
    PT_HIP(hipMemcpyAsync((char*)h->h_out.p + L.work, (char*)h->outbuf.p + L.work, wn,
                          hipMemcpyDeviceToHost, stream));
    PT_HIP(hipStreamSynchronize(stream));
    const uint32_t* hw = (const uint32_t*)(ho + L.work);
    double gram_rows = 0.0, rot_rows = 0.0;
    for (size_t x = 0; x < (size_t)n * L.nslot; ++x) {
      gram_rows += hw[2 * x];
      rot_rows += hw[2 * x + 1];
    }
    const double bw = lo.block_cols;
    const double tiles = bw == 32 ? 10.0 : 3.0;
    pf->st[PTEBD_KERNEL_JACOBI].flops += 2048.0 * tiles * gram_rows + 32.0 * bw * bw * rot_rows;
    pf->st[PTEBD_KERNEL_JACOBI].bytes += ce * (2.0 * bw * gram_rows + 4.0 * bw * rot_rows);
    for (int i = 0; i < n; ++i) {
      const GateDesc& d = descs[i];
      const double cl = d.cl, cm = d.cm, cr = d.cr, kk = hk[i];
      pf->st[PTEBD_KERNEL_THETA].flops += 32.0 * cl * cm * cr + (d.has_gate ? 128.0 * cl * cr : 0.0);
      pf->st[PTEBD_KERNEL_THETA].bytes += ce * (2.0 * cl * cm + 2.0 * cm * cr + 4.0 * cl * cr);
      pf->st[PTEBD_KERNEL_FINALIZE].bytes += ce * (double)(pre ? d.C : d.R) * d.C;
      pf->st[PTEBD_KERNEL_WRITEBACK].bytes += ce * 4.0 * kk * (cl + cr);
      if (pre) {
        // upper-tile FP64 Gram 4 R C^2, Cholesky 8 C^3 / 3, U S = W Yhat 8 R C k
        const double R = d.R, C = d.C;
        pf->st[PTEBD_KERNEL_PRECOND].flops += 4.0 * R * C * C + 8.0 * C * C * C / 3.0 + 8.0 * R * C * kk;
        pf->st[PTEBD_KERNEL_PRECOND].bytes += ce * (3.0 * R * C + 6.0 * C * C + R * kk);
      }
    }
  }
  return PTEBD_OK;
}

int run_updates_dispatch(ptebd_mps* h, const std::vector<Item>& items, double cutoff,
                         int stabilize, int eps_mode, UpdateResult* res) {
  if (h->precision == PTEBD_FP64)
    return run_updates<double>(h, items, cutoff, stabilize, eps_mode, res);
  // FP32 arithmetic leaves rounding residues of up to 2^-20 sigma_1 where an exactly
  // rank-deficient theta has zero singular values; the floor keeps them out of Lambda.
  return run_updates<float>(h, items, std::max(cutoff, PTEBD_FP32_CUTOFF_FLOOR),
                            stabilize, eps_mode, res);
}

int check_handle(ptebd_mps* h) {
  if (!h) return fail(PTEBD_EINVAL, "null handle");
  return PTEBD_OK;
}

int check_state(ptebd_mps* h, int s) {
  PT_CHECK(check_handle(h));
  if (s < 0 || s >= (int)h->st.size()) return fail(PTEBD_EINVAL, "state index out of range");
  return PTEBD_OK;
}

int set_device(ptebd_mps* h) {
  PT_HIP(hipSetDevice(h->device));
  return PTEBD_OK;
}

// Run `steps` PtSU steps on the listed states (each a tSU on all even-q pairs, then all odd).
int run_ptsu(ptebd_mps* h, const std::vector<int>& states, int steps, double cutoff,
             int* max_sweeps, int* n_unconv) {
  for (int step = 0; step < steps; ++step) {
    for (int parity = 0; parity < 2; ++parity) {
      std::vector<Item> items;
      for (int s : states)
        for (int q = parity; q + 1 < h->st[s].n; q += 2) items.push_back({s, q, nullptr, 0});
      UpdateResult res;
      PT_CHECK(run_updates_dispatch(h, items, cutoff, 0, 0, &res));
      *max_sweeps = std::max(*max_sweeps, res.max_sweeps);
      *n_unconv += res.n_unconverged;
    }
  }
  return PTEBD_OK;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// ---------------------------------------------------------------- queries
size_t qscratch_elems(int cap) { return (size_t)cap * cap; }

// Scratch blocks (each cap x cap complex double): E, E2, A0/A1 (2), B0/B1 (2), F0/F1 (2).
struct QScratch {
  cplx<double>* e;
  cplx<double>* e2;
  cplx<double>* a;  // two planes
  cplx<double>* b;  // two planes
  cplx<double>* f;  // two planes
  double* red;      // reduction outputs
};

int get_qscratch(ptebd_mps* h, int cap, QScratch* q, size_t n_red) {
  const size_t blk = qscratch_elems(cap) * sizeof(cplx<double>);
  PT_CHECK(h->qscratch.ensure(blk * 8 + sizeof(double) * n_red + 256));
  char* b = (char*)h->qscratch.p;
  q->e = (cplx<double>*)(b);
  q->e2 = (cplx<double>*)(b + blk);
  q->a = (cplx<double>*)(b + 2 * blk);
  q->b = (cplx<double>*)(b + 4 * blk);
  q->f = (cplx<double>*)(b + 6 * blk);
  q->red = (double*)(b + 8 * blk);
  return PTEBD_OK;
}

// A_s = diag(lam_left) Gamma[q]_s diag(lam_right) of state s of h, in FP64, into out, on
// `stream` (the stream of the query that owns `out`, which may belong to another handle).
void site_a(const ptebd_mps* h, int s, int q, const double* lam_left, const double* lam_right,
            double sl, double sr, cplx<double>* out, hipStream_t stream) {
  const StateInfo& si = h->st[s];
  const int cl = si.dims[q], cm = si.dims[q + 1];
  if (h->precision == PTEBD_FP64)
    ptebd::launch_site_a<double>(h->gamma_slot(s, q), lam_left, lam_right, cl, cm, sl, sr, out,
                                 stream);
  else
    ptebd::launch_site_a<float>(h->gamma_slot(s, q), lam_left, lam_right, cl, cm, sl, sr, out,
                                stream);
}

}  // namespace

namespace ptebd {

int report_error(int code, const char* msg) { return fail(code, msg); }

size_t layer_out_bytes(int n, int cmax) { return out_layout(n, cmax).total; }

LayerOut layer_out_at(void* base, int n, int cmax) {
  return make_layer_out(base, out_layout(n, cmax), cmax);
}

template <class T>
int jacobi_sweeps(hipStream_t stream, const GateDesc* d_desc, int n, int max_c,
                  const LayerOut& lo, int precision, int max_sweeps, double tol_factor,
                  int inner_sweeps, double inner_repeat, int sort_pairs, int32_t* h_counter,
                  int* n_unconverged) {
  return run_jacobi<T>(nullptr, stream, d_desc, n, max_c, lo, precision, max_sweeps, tol_factor,
                       inner_sweeps, inner_repeat, sort_pairs, h_counter, n_unconverged, nullptr);
}

template int jacobi_sweeps<float>(hipStream_t, const GateDesc*, int, int, const LayerOut&, int,
                                  int, double, int, double, int, int32_t*, int*);
template int jacobi_sweeps<double>(hipStream_t, const GateDesc*, int, int, const LayerOut&, int,
                                   int, double, int, double, int, int32_t*, int*);

}  // namespace ptebd

// ============================================================================ C ABI
extern "C" {

const char* ptebd_version(void) { return "ptebd 0.1.0 (gfx950)"; }

const char* ptebd_last_error(void) { return g_last_error.c_str(); }

int ptebd_mps_create(int n_states, const int32_t* n_sites, const int32_t* chi_cap, int d,
                     int precision, void* hip_stream, ptebd_mps_t* out) {
  if (!out) return fail(PTEBD_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_states < 1 || !n_sites || !chi_cap) return fail(PTEBD_EINVAL, "need n_states >= 1 and arrays");
  if (d != 2) return fail(PTEBD_EINVAL, "local dimension d must be 2");
  if (precision == PTEBD_BF16X3)
    return fail(PTEBD_EINVAL, "PTEBD_BF16X3 is not built in this library (use PTEBD_FP32)");
  if (precision != PTEBD_FP64 && precision != PTEBD_FP32)
    return fail(PTEBD_EINVAL, "precision must be PTEBD_FP64 or PTEBD_FP32");
  for (int s = 0; s < n_states; ++s) {
    if (n_sites[s] < 2) return fail(PTEBD_EINVAL, "every state needs n_sites >= 2");
    if (chi_cap[s] < 1 || chi_cap[s] > 512) return fail(PTEBD_EINVAL, "chi_cap must be in [1, 512]");
  }
  ptebd_mps* h = new (std::nothrow) ptebd_mps();
  if (!h) return fail(PTEBD_ENOMEM, "host allocation failed");
  auto cleanup = [&](int code) {
    ptebd_mps_destroy(h);
    return code;
  };
  if (hipGetDevice(&h->device) != hipSuccess) return cleanup(fail(PTEBD_EDEVICE, "no HIP device"));
  h->stream = (hipStream_t)hip_stream;
  h->precision = precision;
  // measured at chi = 256 (one saturated layer): FP32 fastest with 2 inner sweeps, FP64
  // with 1 (the FP64 inner sweep costs more than the outer sweeps it saves)
  h->inner_sweeps = precision == PTEBD_FP64 ? 1 : 2;
  h->inner_repeat = precision == PTEBD_FP64 ? 0.0 : 1e-2;
  // FP32: pairs orthogonal to u sqrt(R) (tol_factor 1).  Measured at chi = 256 (N = 1024,
  // Haar SU(4), 34 layers): against the FP64 path err_F is 5x smaller than with 4 u sqrt(R)
  // at every depth for 2 % more sweeps; below 1 the rounding of the cosines leaves SVDs
  // unconverged.  FP64 keeps 4 u sqrt(R), orders of magnitude inside its budget.
  h->tol_factor = precision == PTEBD_FP64 ? 4.0 : 1.0;
  h->celem = precision == PTEBD_FP64 ? sizeof(cplx<double>) : sizeof(cplx<float>);
  size_t goff = 0, loff = 0;
  h->st.resize(n_states);
  int total_sites = 0, total_bonds = 0;
  for (int s = 0; s < n_states; ++s) {
    StateInfo& si = h->st[s];
    si.n = n_sites[s];
    si.cap = chi_cap[s];
    si.dims.assign(si.n + 1, 1);
    si.gamma_off = goff;
    si.lam_off = loff;
    goff += (size_t)si.n * 2 * si.cap * si.cap;
    loff += (size_t)(si.n + 1) * si.cap;
    total_sites += si.n;
    total_bonds += si.n + 1;
  }
  int st = h->gamma.ensure(goff * h->celem);
  if (st < 0) return cleanup(st);
  st = h->lam.ensure(loff * sizeof(double));
  if (st < 0) return cleanup(st);
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess)
    return cleanup(fail(PTEBD_EDEVICE, "hipEventCreate failed"));
  std::vector<size_t> go, lo;
  for (int s = 0; s < n_states; ++s) {
    const StateInfo& si = h->st[s];
    for (int q = 0; q < si.n; ++q) go.push_back((si.gamma_off + (size_t)q * 2 * si.cap * si.cap) * h->celem);
    for (int i = 0; i <= si.n; ++i) lo.push_back(si.lam_off + (size_t)i * si.cap);
  }
  DevBuf offs;
  st = offs.ensure(sizeof(size_t) * (go.size() + lo.size()));
  if (st < 0) return cleanup(st);
  size_t* d_go = (size_t*)offs.p;
  size_t* d_lo = d_go + go.size();
  if (hipMemcpyAsync(d_go, go.data(), sizeof(size_t) * go.size(), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipMemcpyAsync(d_lo, lo.data(), sizeof(size_t) * lo.size(), hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return cleanup(fail(PTEBD_EDEVICE, "copy of slot offsets failed"));
  if (precision == PTEBD_FP64)
    ptebd::launch_init_product<double>(h->gamma.p, d_go, total_sites, (double*)h->lam.p, d_lo,
                                       total_bonds, h->stream);
  else
    ptebd::launch_init_product<float>(h->gamma.p, d_go, total_sites, (double*)h->lam.p, d_lo,
                                      total_bonds, h->stream);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) {
    offs.release();
    return cleanup(fail(PTEBD_EDEVICE, "initialization of |0...0> failed"));
  }
  offs.release();
  *out = h;
  return PTEBD_OK;
}

int ptebd_mps_destroy(ptebd_mps_t h) {
  if (!h) return PTEBD_OK;
  (void)hipStreamSynchronize(h->stream);
  h->gamma.release();
  h->lam.release();
  h->work.release();
  h->desc.release();
  h->gates.release();
  h->outbuf.release();
  h->qscratch.release();
  h->renv.release();
  h->qout.release();
  h->aux.release();
  h->samp.release();
  h->h_desc.release();
  h->h_gates.release();
  h->h_out.release();
  h->h_small.release();
  h->prof.release();
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  if (h->stream2) {
    (void)hipStreamSynchronize(h->stream2);
    (void)hipStreamDestroy(h->stream2);
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  for (auto& evs : h->ev_sweep)
    for (hipEvent_t e : evs)
      if (e) (void)hipEventDestroy(e);
  h->sweep_graphs.release();
  delete h;
  return PTEBD_OK;
}

int ptebd_get_svd_params(ptebd_mps_t h, ptebd_svd_params* out) {
  PT_CHECK(check_handle(h));
  if (!out) return fail(PTEBD_EINVAL, "params is NULL");
  out->max_sweeps = h->max_sweeps;
  out->tol_factor = h->tol_factor;
  out->inner_sweeps = h->inner_sweeps;
  out->inner_repeat = h->inner_repeat;
  out->sort_pairs = h->sort_pairs;
  out->precondition = h->precondition;
  out->streams = h->streams;
  out->block_cols = h->block_cols;
  out->graphs = h->graphs;
  return PTEBD_OK;
}

int ptebd_set_svd_params(ptebd_mps_t h, const ptebd_svd_params* p) {
  PT_CHECK(check_handle(h));
  if (!p) return fail(PTEBD_EINVAL, "params is NULL");
  if (p->max_sweeps < 1 || !(p->tol_factor > 0.0) || !std::isfinite(p->tol_factor) ||
      p->inner_sweeps < 1 || p->inner_sweeps > 64 || !(p->inner_repeat >= 0.0) ||
      !std::isfinite(p->inner_repeat) || (p->sort_pairs != 0 && p->sort_pairs != 1) ||
      (p->precondition != 0 && p->precondition != 1) || (p->streams != 1 && p->streams != 2) ||
      (p->block_cols != 16 && p->block_cols != 32) ||
      (p->block_cols == 32 && h->precision != PTEBD_FP32) || (p->graphs != 0 && p->graphs != 1))
    return fail(PTEBD_EINVAL, "need max_sweeps >= 1, tol_factor > 0, inner_sweeps in [1, 64], "
                              "finite inner_repeat >= 0, sort_pairs, precondition and graphs "
                              "0/1, streams 1 or 2, block_cols 16 or (FP32 only) 32");
  h->max_sweeps = p->max_sweeps;
  h->tol_factor = p->tol_factor;
  h->inner_sweeps = p->inner_sweeps;
  h->inner_repeat = p->inner_repeat;
  h->sort_pairs = p->sort_pairs;
  h->precondition = p->precondition;
  h->streams = p->streams;
  h->block_cols = p->block_cols;
  h->graphs = p->graphs;
  return PTEBD_OK;
}

int ptebd_apply_layer(ptebd_mps_t h, int n_gates, const int32_t* state_idx,
                      const int32_t* bonds, const double* gates, int chi_max, double cutoff,
                      int ptsu_steps, int flags, ptebd_layer_stats* stats) {
  PT_CHECK(check_handle(h));
  if (n_gates < 0) return fail(PTEBD_EINVAL, "n_gates < 0");
  if (n_gates > 0 && (!bonds || !gates)) return fail(PTEBD_EINVAL, "bonds / gates are NULL");
  if (!state_idx && h->st.size() != 1 && n_gates > 0)
    return fail(PTEBD_EINVAL, "state_idx may be NULL only for a single-state handle");
  if (!(cutoff >= 0.0) || !(cutoff < 1.0)) return fail(PTEBD_EINVAL, "cutoff must be in [0, 1)");
  if (ptsu_steps < 0) return fail(PTEBD_EINVAL, "ptsu_steps < 0");
  if (flags & ~(PTEBD_FLAG_NO_STABILIZE | PTEBD_FLAG_RELATIVE_EPS | PTEBD_FLAG_COMPLEMENT_EPS))
    return fail(PTEBD_EINVAL, "unknown flags");
  if ((flags & PTEBD_FLAG_RELATIVE_EPS) && (flags & PTEBD_FLAG_COMPLEMENT_EPS))
    return fail(PTEBD_EINVAL, "RELATIVE_EPS and COMPLEMENT_EPS exclude each other");
  if (chi_max < 0) return fail(PTEBD_EINVAL, "chi_max must be >= 0");
  std::vector<std::vector<char>> used(h->st.size());
  std::vector<Item> items(n_gates);
  for (int i = 0; i < n_gates; ++i) {
    const int s = state_idx ? state_idx[i] : 0;
    if (s < 0 || s >= (int)h->st.size()) return fail(PTEBD_EINVAL, "state index out of range");
    const StateInfo& si = h->st[s];
    if (chi_max > si.cap) return fail(PTEBD_EINVAL, "chi_max exceeds the state's chi_cap");
    const int chi = chi_max > 0 ? chi_max : si.cap;
    const int q = bonds[i];
    if (q < 0 || q + 1 >= si.n) return fail(PTEBD_EINVAL, "bond q out of range");
    if (used[s].empty()) used[s].assign(si.n, 0);
    if (used[s][q] || used[s][q + 1])
      return fail(PTEBD_EOVERLAP, "gates overlap at site " + std::to_string(q) + " of state " + std::to_string(s));
    used[s][q] = used[s][q + 1] = 1;
    if (!finite_all(gates + 32 * (size_t)i, 32)) return fail(PTEBD_EINVAL, "non-finite gate entry");
    // the new bond must fit the slot: min(2 chi_q, 2 chi_{q+2}) is capped by chi_max
    items[i] = {s, q, gates + 32 * (size_t)i, chi};
  }
  PT_CHECK(set_device(h));
  PT_HIP(hipEventRecord(h->ev0, h->stream));
  UpdateResult res;
  PT_CHECK(run_updates_dispatch(h, items, cutoff,
                                (flags & PTEBD_FLAG_NO_STABILIZE) ? 0 : 1,
                                (flags & PTEBD_FLAG_RELATIVE_EPS)     ? 1
                                : (flags & PTEBD_FLAG_COMPLEMENT_EPS) ? 2
                                                                      : 0,
                                &res));
  std::vector<int> trig_states;
  std::vector<char> trig(h->st.size(), 0);
  for (int i = 0; i < n_gates; ++i)
    if (res.r[i] > items[i].chi) trig[items[i].s] = 1;
  for (size_t s = 0; s < trig.size(); ++s)
    if (trig[s]) trig_states.push_back((int)s);
  for (int i = 0; i < n_gates; ++i) {
    StateInfo& si = h->st[items[i].s];
    si.prod_nu *= res.nu[i];
    si.prod_fid *= (1.0 - res.eps[i]);
  }
  int max_sw = res.max_sweeps, n_unconv = res.n_unconverged, ptsu_done = 0;
  if (ptsu_steps > 0 && !trig_states.empty()) {
    PT_CHECK(run_ptsu(h, trig_states, ptsu_steps, cutoff, &max_sw, &n_unconv));
    ptsu_done = ptsu_steps;
  }
  PT_HIP(hipEventRecord(h->ev1, h->stream));
  PT_HIP(hipEventSynchronize(h->ev1));
  float ms = 0.f;
  PT_HIP(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  if (stats) {
    for (int i = 0; i < n_gates; ++i) {
      if (stats->k) stats->k[i] = res.k[i];
      if (stats->rank) stats->rank[i] = res.r[i];
      if (stats->eps) stats->eps[i] = res.eps[i];
      if (stats->nu) stats->nu[i] = res.nu[i];
      if (stats->sweeps) stats->sweeps[i] = res.sweeps[i];
    }
    stats->triggered = trig_states.empty() ? 0 : 1;
    stats->ptsu_done = ptsu_done;
    stats->max_sweeps = max_sw;
    stats->n_unconverged = n_unconv;
    stats->device_ms = ms;
  }
  if (n_unconv > 0) return fail(PTEBD_WNOCONV, "some SVDs reached the sweep cap");
  return PTEBD_OK;
}

int ptebd_set_profiling(ptebd_mps_t h, int enable) {
  PT_CHECK(check_handle(h));
  PT_HIP(hipStreamSynchronize(h->stream));
  h->prof.harvest();
  h->prof.reset();
  h->prof.on = enable != 0;
  return PTEBD_OK;
}

int ptebd_get_kernel_stats(ptebd_mps_t h, int kind, ptebd_kernel_stats* out) {
  PT_CHECK(check_handle(h));
  if (kind < 0 || kind >= PTEBD_KERNEL_COUNT || !out) return fail(PTEBD_EINVAL, "bad kernel class");
  PT_HIP(hipStreamSynchronize(h->stream));
  h->prof.harvest();
  *out = h->prof.st[kind];
  return PTEBD_OK;
}

int ptebd_canonicalize(ptebd_mps_t h, int s, double cutoff, double* norm_out) {
  PT_CHECK(check_state(h, s));
  if (!(cutoff >= 0.0) || !(cutoff < 1.0)) return fail(PTEBD_EINVAL, "cutoff must be in [0, 1)");
  PT_CHECK(set_device(h));
  const int n = h->st[s].n;
  int n_unconv = 0;
  // Sweeps from both ends.  Bonds q = 0 .. n-2 (a tSU at q acts on sites q, q+1); m is the
  // middle bond.  Pass 1 sweeps q = 0, 1, .., m-1 (left block left-canonical) and, in the
  // same batch, q = n-2, n-3, .., m+1 (right block right-canonical); the tSU at m then sees
  // identity environments on both sides and gives the exact Schmidt decomposition there;
  // pass 2 sweeps q = m-1, .., 0 and q = m+1, .., n-2 together.  The two items of a batch
  // act on disjoint sites and share only a read of Lambda[m+1]; a tSU inside one block only
  // regauges that block's interior, so the other block's environment stays the identity.
  // About n sequential steps instead of the 2(n-1) of one sweep there and one back.
  const int m = (n - 2) / 2;
  // Each step is a batch of one or two SVDs, so a Jacobi round lasts as long as one
  // workgroup's inner Jacobi: one inner sweep per pair (the outer convergence test is
  // unchanged) costs more rounds but less time (N = 256, chi = 256: 2.84 s against 3.11 s).
  struct InnerSweeps {
    ptebd_mps* h;
    int saved;
    ~InnerSweeps() { h->inner_sweeps = saved; }
  } inner_guard{h, h->inner_sweeps};
  h->inner_sweeps = 1;
  auto step = [&](int ql, int qr) -> int {
    std::vector<Item> items;
    if (ql >= 0) items.push_back(Item{s, ql, nullptr, 0});
    if (qr >= 0) items.push_back(Item{s, qr, nullptr, 0});
    if (items.empty()) return PTEBD_OK;
    UpdateResult res;
    PT_CHECK(run_updates_dispatch(h, items, cutoff, 0, 0, &res));
    n_unconv += res.n_unconverged;
    return PTEBD_OK;
  };
  if (n >= 2) {
    const int span = std::max(m, n - 2 - m);
    for (int t = 0; t < span; ++t)
      PT_CHECK(step(t < m ? t : -1, n - 2 - t > m ? n - 2 - t : -1));
    PT_CHECK(step(m, -1));
    for (int t = 0; t < span; ++t)
      PT_CHECK(step(m - 1 - t >= 0 ? m - 1 - t : -1, m + 1 + t <= n - 2 ? m + 1 + t : -1));
  }
  const StateInfo& si = h->st[s];
  // in canonical form every bond carries the whole norm: n^2 = sum Lambda[1]^2
  std::vector<double> l1(si.dims[1]);
  PT_HIP(hipStreamSynchronize(h->stream));
  PT_HIP(hipMemcpy(l1.data(), h->lam_slot(s, 1), sizeof(double) * l1.size(),
                   hipMemcpyDeviceToHost));
  double n2 = 0.0;
  for (double v : l1) n2 += v * v;
  const double nrm = std::sqrt(n2);
  if (!(nrm > 0.0) || !std::isfinite(nrm))
    return fail(PTEBD_ENONFINITE, "canonicalize: the state norm is zero or not finite");
  PT_CHECK(h->aux.ensure(sizeof(int32_t) * (si.n + 1)));
  PT_HIP(hipMemcpyAsync(h->aux.p, si.dims.data(), sizeof(int32_t) * (si.n + 1),
                        hipMemcpyHostToDevice, h->stream));
  int max_elems = 1;
  for (int q = 0; q < si.n; ++q) max_elems = std::max(max_elems, 2 * si.dims[q] * si.dims[q + 1]);
  const size_t slot = 2 * (size_t)si.cap * si.cap;
  if (h->precision == PTEBD_FP64)
    ptebd::launch_scale_state<double>(h->gamma_slot(s, 0), slot, h->lam_slot(s, 0), si.cap,
                                      (const int32_t*)h->aux.p, si.n, max_elems, nrm, h->stream);
  else
    ptebd::launch_scale_state<float>(h->gamma_slot(s, 0), slot, h->lam_slot(s, 0), si.cap,
                                     (const int32_t*)h->aux.p, si.n, max_elems, nrm, h->stream);
  PT_HIP(hipGetLastError());
  PT_HIP(hipStreamSynchronize(h->stream));
  if (norm_out) *norm_out = nrm;
  if (n_unconv > 0) return fail(PTEBD_WNOCONV, "some SVDs reached the sweep cap");
  return PTEBD_OK;
}

int ptebd_sample(ptebd_mps_t h, int s, int n_samples, const double* uniforms, uint8_t* bits) {
  PT_CHECK(check_state(h, s));
  if (n_samples < 0) return fail(PTEBD_EINVAL, "n_samples < 0");
  if (n_samples == 0) return PTEBD_OK;
  if (!uniforms || !bits) return fail(PTEBD_EINVAL, "uniforms / bits are NULL");
  const StateInfo& si = h->st[s];
  const int n = si.n;
  const size_t cnt = (size_t)n_samples * n;
  for (size_t e = 0; e < cnt; ++e)
    if (!(uniforms[e] >= 0.0 && uniforms[e] < 1.0))
      return fail(PTEBD_EINVAL, "uniforms must lie in [0, 1)");
  PT_CHECK(set_device(h));
  // device layout: uniforms | bits | W ping-pong | sel ping-pong | scale ping-pong | err |
  // partial norms per sample and column tile
  const int ldw = 2 * si.cap;
  const int max_tiles = (ldw + 31) / 32;
  const size_t wbytes = h->celem * (size_t)n_samples * ldw;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_u = 0, o_b = al(o_u + sizeof(double) * cnt), o_w0 = al(o_b + cnt),
               o_w1 = al(o_w0 + wbytes), o_s0 = al(o_w1 + wbytes),
               o_s1 = al(o_s0 + sizeof(int32_t) * n_samples),
               o_c0 = al(o_s1 + sizeof(int32_t) * n_samples),
               o_c1 = al(o_c0 + sizeof(double) * n_samples),
               o_e = al(o_c1 + sizeof(double) * n_samples), o_p = o_e + 256,
               total = o_p + sizeof(double) * 2 * (size_t)n_samples * max_tiles;
  PT_CHECK(h->samp.ensure(total));
  char* base = (char*)h->samp.p;
  PT_HIP(hipMemcpyAsync(base + o_u, uniforms, sizeof(double) * cnt, hipMemcpyHostToDevice,
                        h->stream));
  PT_HIP(hipMemsetAsync(base + o_e, 0, sizeof(int32_t), h->stream));
  Prof* pf = &h->prof;
  for (int q = 0; q < n; ++q) {
    const int cur = q & 1;
    ptebd::SampleSite a;
    a.gamma = h->gamma_slot(s, q);
    a.lam_r = h->lam_slot(s, q + 1);
    a.cl = si.dims[q];
    a.cm = si.dims[q + 1];
    a.first = q == 0;
    a.n_samples = n_samples;
    a.ldw = ldw;
    a.w_in = base + (cur ? o_w0 : o_w1);
    a.w_out = base + (cur ? o_w1 : o_w0);
    a.sel_in = (const int32_t*)(base + (cur ? o_s0 : o_s1));
    a.scale_in = (const double*)(base + (cur ? o_c0 : o_c1));
    a.sel_out = (int32_t*)(base + (cur ? o_s1 : o_s0));
    a.scale_out = (double*)(base + (cur ? o_c1 : o_c0));
    a.u = (const double*)(base + o_u) + q;
    a.ustride = n;
    a.bits = (uint8_t*)(base + o_b) + q;
    a.bstride = n;
    a.err = (int32_t*)(base + o_e);
    a.part = (double*)(base + o_p);
    a.ntiles = (2 * a.cm + 31) / 32;
    timed(pf, PTEBD_KERNEL_SAMPLE, h->stream, [&] {
      if (h->precision == PTEBD_FP64)
        ptebd::launch_sample_site<double>(a, h->stream);
      else
        ptebd::launch_sample_site<float>(a, h->stream);
    });
    if (pf->on) {
      const double ce = (double)h->celem;
      pf->st[PTEBD_KERNEL_SAMPLE].flops += 16.0 * n_samples * (double)a.cl * a.cm;
      pf->st[PTEBD_KERNEL_SAMPLE].bytes +=
          ce * (2.0 * a.cl * a.cm + (double)n_samples * (a.cl + 2.0 * a.cm));
    }
  }
  PT_HIP(hipGetLastError());
  int32_t err = 0;
  PT_HIP(hipMemcpyAsync(bits, base + o_b, cnt, hipMemcpyDeviceToHost, h->stream));
  PT_HIP(hipMemcpyAsync(&err, base + o_e, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  PT_HIP(hipStreamSynchronize(h->stream));
  if (pf->on) pf->harvest();
  if (err) return fail(PTEBD_ENONFINITE, "a conditional probability vanished (state not canonical?)");
  return PTEBD_OK;
}

int ptebd_ptsu(ptebd_mps_t h, int s, int steps, double cutoff) {
  PT_CHECK(check_state(h, s));
  if (steps < 0) return fail(PTEBD_EINVAL, "steps < 0");
  if (!(cutoff >= 0.0) || !(cutoff < 1.0)) return fail(PTEBD_EINVAL, "cutoff must be in [0, 1)");
  PT_CHECK(set_device(h));
  int ms = 0, nu = 0;
  PT_CHECK(run_ptsu(h, std::vector<int>{s}, steps, cutoff, &ms, &nu));
  if (nu > 0) return fail(PTEBD_WNOCONV, "some SVDs reached the sweep cap");
  return PTEBD_OK;
}

int ptebd_overlap(ptebd_mps_t ha, int sa, ptebd_mps_t hb, int sb, double* re, double* im) {
  PT_CHECK(check_state(ha, sa));
  PT_CHECK(check_state(hb, sb));
  if (!re || !im) return fail(PTEBD_EINVAL, "null output");
  const StateInfo& A = ha->st[sa];
  const StateInfo& B = hb->st[sb];
  if (A.n != B.n) return fail(PTEBD_EINVAL, "states differ in the number of sites");
  if (ha->device != hb->device) return fail(PTEBD_EINVAL, "handles live on different devices");
  PT_CHECK(set_device(ha));
  // hb's pending work has completed; from here on every kernel, hb's site tensors included,
  // runs on ha's stream, which orders them against the scratch buffers they share
  PT_HIP(hipStreamSynchronize(hb->stream));
  const int cap = std::max(A.cap, B.cap);
  QScratch q;
  PT_CHECK(get_qscratch(ha, cap, &q, 4));
  hipStream_t stream = ha->stream;
  ptebd::launch_set_identity_scalar(q.e, 1.0, stream);
  const size_t blk = qscratch_elems(cap);
  for (int site = 0; site < A.n; ++site) {
    const int cla = A.dims[site], cma = A.dims[site + 1];
    const int clb = B.dims[site], cmb = B.dims[site + 1];
    site_a(ha, sa, site, ha->lam_slot(sa, site), nullptr, 1.0, 1.0, q.a, stream);
    site_a(hb, sb, site, hb->lam_slot(sb, site), nullptr, 1.0, 1.0, q.b, stream);
    // F_s = E B_s : (cla x clb)(clb x cmb)
    for (int s = 0; s < 2; ++s)
      ptebd::launch_zgemm('N', 'N', cla, cmb, clb, 1.0, q.e, cla, q.b + (size_t)s * clb * cmb, clb,
                          0.0, q.f + s * blk, cla, stream);
    // E' = sum_s A_s^H F_s : (cma x cla)(cla x cmb)
    for (int s = 0; s < 2; ++s)
      ptebd::launch_zgemm('C', 'N', cma, cmb, cla, 1.0, q.a + (size_t)s * cla * cma, cla,
                          q.f + s * blk, cla, s == 0 ? 0.0 : 1.0, q.e2, cma, stream);
    std::swap(q.e, q.e2);
  }
  PT_HIP(hipGetLastError());
  cplx<double> hv;
  PT_HIP(hipMemcpyAsync(&hv, q.e, sizeof(hv), hipMemcpyDeviceToHost, stream));
  PT_HIP(hipStreamSynchronize(stream));
  // Lambda[N] = (1) for both states
  *re = hv.re;
  *im = hv.im;
  return PTEBD_OK;
}

int ptebd_norm(ptebd_mps_t h, int s, double* out) {
  if (!out) return fail(PTEBD_EINVAL, "null output");
  double re = 0, im = 0;
  PT_CHECK(ptebd_overlap(h, s, h, s, &re, &im));
  *out = std::sqrt(std::max(re, 0.0));
  return PTEBD_OK;
}

int ptebd_expect_z(ptebd_mps_t h, int s, double* out) {
  PT_CHECK(check_state(h, s));
  if (!out) return fail(PTEBD_EINVAL, "null output");
  PT_CHECK(set_device(h));
  const StateInfo& si = h->st[s];
  const int n = si.n, cap = si.cap;
  const size_t blk = qscratch_elems(cap);
  QScratch q;
  PT_CHECK(get_qscratch(h, cap, &q, (size_t)n + 4));
  PT_CHECK(h->renv.ensure(sizeof(cplx<double>) * blk * (size_t)(n + 1)));
  cplx<double>* renv = (cplx<double>*)h->renv.p;
  hipStream_t stream = h->stream;
  PT_HIP(hipMemsetAsync(q.red, 0, sizeof(double) * (n + 4), stream));
  // right environments R[q] = sum_s A_s R[q+1] A_s^H, R[N] = (1)
  ptebd::launch_set_identity_scalar(renv + (size_t)n * blk, 1.0, stream);
  for (int site = n - 1; site >= 0; --site) {
    const int cl = si.dims[site], cm = si.dims[site + 1];
    site_a(h, s, site, h->lam_slot(s, site), nullptr, 1.0, 1.0, q.a, stream);
    for (int p = 0; p < 2; ++p)
      ptebd::launch_zgemm('N', 'N', cl, cm, cm, 1.0, q.a + (size_t)p * cl * cm, cl,
                          renv + (size_t)(site + 1) * blk, cm, 0.0, q.f + p * blk, cl, stream);
    for (int p = 0; p < 2; ++p)
      ptebd::launch_zgemm('N', 'C', cl, cl, cm, 1.0, q.f + p * blk, cl, q.a + (size_t)p * cl * cm,
                          cl, p == 0 ? 0.0 : 1.0, renv + (size_t)site * blk, cl, stream);
  }
  // left sweep with <Z_q> on the fly: z_q = sum_s z_s Tr(A_s^H L A_s R[q+1])
  ptebd::launch_set_identity_scalar(q.e, 1.0, stream);
  for (int site = 0; site < n; ++site) {
    const int cl = si.dims[site], cm = si.dims[site + 1];
    site_a(h, s, site, h->lam_slot(s, site), nullptr, 1.0, 1.0, q.a, stream);
    for (int p = 0; p < 2; ++p) {
      // F_p = L A_p (cl x cm)
      ptebd::launch_zgemm('N', 'N', cl, cm, cl, 1.0, q.e, cl, q.a + (size_t)p * cl * cm, cl, 0.0,
                          q.f + p * blk, cl, stream);
      // B_p = F_p R[q+1] (cl x cm), stored in q.b planes
      ptebd::launch_zgemm('N', 'N', cl, cm, cm, 1.0, q.f + p * blk, cl,
                          renv + (size_t)(site + 1) * blk, cm, 0.0, q.b + p * blk, cl, stream);
      ptebd::launch_dot_conj(q.a + (size_t)p * cl * cm, q.b + p * blk, cl * cm, p == 0 ? 1.0 : -1.0,
                             q.red + site, stream);
    }
    // L' = sum_p A_p^H F_p (cm x cm)
    for (int p = 0; p < 2; ++p)
      ptebd::launch_zgemm('C', 'N', cm, cm, cl, 1.0, q.a + (size_t)p * cl * cm, cl, q.f + p * blk,
                          cl, p == 0 ? 0.0 : 1.0, q.e2, cm, stream);
    std::swap(q.e, q.e2);
  }
  PT_HIP(hipGetLastError());
  std::vector<double> z(n);
  cplx<double> nrm;
  PT_HIP(hipMemcpyAsync(z.data(), q.red, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
  PT_HIP(hipMemcpyAsync(&nrm, q.e, sizeof(nrm), hipMemcpyDeviceToHost, stream));
  PT_HIP(hipStreamSynchronize(stream));
  for (int i = 0; i < n; ++i) out[i] = z[i] / nrm.re;
  return PTEBD_OK;
}

int ptebd_canon_distance(ptebd_mps_t h, int s, double* out) {
  PT_CHECK(check_state(h, s));
  if (!out) return fail(PTEBD_EINVAL, "null output");
  double nrm = 0;
  PT_CHECK(ptebd_norm(h, s, &nrm));
  if (!(nrm > 0)) return fail(PTEBD_EANNIHILATED, "zero norm");
  const StateInfo& si = h->st[s];
  const int n = si.n, cap = si.cap;
  const double scale = std::pow(nrm, -1.0 / (n - 1));
  QScratch q;
  PT_CHECK(get_qscratch(h, cap, &q, (size_t)2 * n));
  hipStream_t stream = h->stream;
  const size_t blk = qscratch_elems(cap);
  for (int site = 0; site < n; ++site) {
    const int cl = si.dims[site], cm = si.dims[site + 1];
    const double sl = (site >= 1) ? scale : 1.0;
    const double sr = (site + 1 <= n - 1) ? scale : 1.0;
    // A = Lambda[q] Gamma[q] and B = Gamma[q] Lambda[q+1] with the inner Lambdas scaled
    site_a(h, s, site, h->lam_slot(s, site), nullptr, sl, 1.0, q.a, stream);
    site_a(h, s, site, nullptr, h->lam_slot(s, site + 1), 1.0, sr, q.b, stream);
    for (int p = 0; p < 2; ++p)
      ptebd::launch_zgemm('C', 'N', cm, cm, cl, 1.0, q.a + (size_t)p * cl * cm, cl,
                          q.a + (size_t)p * cl * cm, cl, p == 0 ? 0.0 : 1.0, q.e, cm, stream);
    ptebd::launch_frob_minus_identity(q.e, cm, q.red + 2 * site, stream);
    for (int p = 0; p < 2; ++p)
      ptebd::launch_zgemm('N', 'C', cl, cl, cm, 1.0, q.b + (size_t)p * cl * cm, cl,
                          q.b + (size_t)p * cl * cm, cl, p == 0 ? 0.0 : 1.0, q.e2, cl, stream);
    ptebd::launch_frob_minus_identity(q.e2, cl, q.red + 2 * site + 1, stream);
  }
  (void)blk;
  PT_HIP(hipGetLastError());
  std::vector<double> red(2 * (size_t)n);
  PT_HIP(hipMemcpyAsync(red.data(), q.red, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, stream));
  PT_HIP(hipStreamSynchronize(stream));
  double total = 0;
  for (int i = 0; i < 2 * n; ++i) total += std::sqrt(red[i]);
  *out = total / (2.0 * n);
  return PTEBD_OK;
}

int ptebd_norm_estimate(ptebd_mps_t h, int s, double* out) {
  PT_CHECK(check_state(h, s));
  if (!out) return fail(PTEBD_EINVAL, "null output");
  *out = h->st[s].prod_nu;
  return PTEBD_OK;
}

int ptebd_fidelity_estimate(ptebd_mps_t h, int s, double* out) {
  PT_CHECK(check_state(h, s));
  if (!out) return fail(PTEBD_EINVAL, "null output");
  *out = h->st[s].prod_fid;
  return PTEBD_OK;
}

int ptebd_bond_dims(ptebd_mps_t h, int s, int32_t* out, int cap) {
  PT_CHECK(check_state(h, s));
  const StateInfo& si = h->st[s];
  if (!out || cap < si.n + 1) return fail(PTEBD_EINVAL, "output too small");
  for (int i = 0; i <= si.n; ++i) out[i] = si.dims[i];
  return PTEBD_OK;
}

int ptebd_get_lambda(ptebd_mps_t h, int s, int bond, double* out, int cap, int* len) {
  PT_CHECK(check_state(h, s));
  const StateInfo& si = h->st[s];
  if (bond < 0 || bond > si.n) return fail(PTEBD_EINVAL, "bond out of range");
  const int chi = si.dims[bond];
  if (len) *len = chi;
  if (!out || cap < chi) return fail(PTEBD_EINVAL, "output too small");
  PT_CHECK(set_device(h));
  PT_HIP(hipMemcpyAsync(out, h->lam_slot(s, bond), sizeof(double) * chi, hipMemcpyDeviceToHost,
                        h->stream));
  PT_HIP(hipStreamSynchronize(h->stream));
  return PTEBD_OK;
}

int ptebd_export(ptebd_mps_t h, int s, double* gamma, size_t gamma_cap, double* lambda,
                 size_t lambda_cap) {
  PT_CHECK(check_state(h, s));
  const StateInfo& si = h->st[s];
  size_t need_g = 0, need_l = 0;
  for (int q = 0; q < si.n; ++q) need_g += 2 * 2 * (size_t)si.dims[q] * si.dims[q + 1];
  for (int i = 0; i <= si.n; ++i) need_l += si.dims[i];
  if (!gamma || !lambda || gamma_cap < need_g || lambda_cap < need_l)
    return fail(PTEBD_EINVAL, "export buffers too small");
  PT_CHECK(set_device(h));
  PT_HIP(hipStreamSynchronize(h->stream));
  std::vector<char> tmp;
  size_t go = 0, lo = 0;
  for (int q = 0; q < si.n; ++q) {
    const int cl = si.dims[q], cm = si.dims[q + 1];
    const size_t cnt = 2 * (size_t)cl * cm;
    tmp.resize(cnt * h->celem);
    PT_HIP(hipMemcpy(tmp.data(), h->gamma_slot(s, q), cnt * h->celem, hipMemcpyDeviceToHost));
    for (int a = 0; a < cl; ++a)
      for (int p = 0; p < 2; ++p)
        for (int m = 0; m < cm; ++m) {
          const size_t src = (size_t)p * cl * cm + (size_t)m * cl + a;
          const size_t dst = go + 2 * (((size_t)a * 2 + p) * cm + m);
          if (h->precision == PTEBD_FP64) {
            const cplx<double> z = ((const cplx<double>*)tmp.data())[src];
            gamma[dst] = z.re;
            gamma[dst + 1] = z.im;
          } else {
            const cplx<float> z = ((const cplx<float>*)tmp.data())[src];
            gamma[dst] = z.re;
            gamma[dst + 1] = z.im;
          }
        }
    go += 2 * cnt;
  }
  for (int i = 0; i <= si.n; ++i) {
    PT_HIP(hipMemcpy(lambda + lo, h->lam_slot(s, i), sizeof(double) * si.dims[i], hipMemcpyDeviceToHost));
    lo += si.dims[i];
  }
  return PTEBD_OK;
}

int ptebd_export_site(ptebd_mps_t h, int s, int q, double* gamma, size_t gamma_cap,
                      int32_t* dims_out) {
  PT_CHECK(check_state(h, s));
  const StateInfo& si = h->st[s];
  if (q < 0 || q >= si.n) return fail(PTEBD_EINVAL, "site out of range");
  const int cl = si.dims[q], cm = si.dims[q + 1];
  const size_t cnt = 2 * (size_t)cl * cm;
  if (!gamma || gamma_cap < 2 * cnt) return fail(PTEBD_EINVAL, "export buffer too small");
  PT_CHECK(set_device(h));
  PT_HIP(hipStreamSynchronize(h->stream));
  std::vector<char> tmp(cnt * h->celem);
  PT_HIP(hipMemcpy(tmp.data(), h->gamma_slot(s, q), cnt * h->celem, hipMemcpyDeviceToHost));
  for (int a = 0; a < cl; ++a)
    for (int p = 0; p < 2; ++p)
      for (int m = 0; m < cm; ++m) {
        const size_t src = (size_t)p * cl * cm + (size_t)m * cl + a;
        const size_t dst = 2 * (((size_t)a * 2 + p) * cm + m);
        if (h->precision == PTEBD_FP64) {
          const cplx<double> z = ((const cplx<double>*)tmp.data())[src];
          gamma[dst] = z.re;
          gamma[dst + 1] = z.im;
        } else {
          const cplx<float> z = ((const cplx<float>*)tmp.data())[src];
          gamma[dst] = z.re;
          gamma[dst + 1] = z.im;
        }
      }
  if (dims_out) {
    dims_out[0] = cl;
    dims_out[1] = cm;
  }
  return PTEBD_OK;
}

int ptebd_import(ptebd_mps_t h, int s, const int32_t* dims, const double* gamma,
                 const double* lambda) {
  PT_CHECK(check_state(h, s));
  StateInfo& si = h->st[s];
  if (!dims || !gamma || !lambda) return fail(PTEBD_EINVAL, "null input");
  if (dims[0] != 1 || dims[si.n] != 1) return fail(PTEBD_EINVAL, "chi_0 and chi_N must be 1");
  size_t need_g = 0, need_l = 0;
  for (int i = 0; i <= si.n; ++i) {
    if (dims[i] < 1 || dims[i] > si.cap) return fail(PTEBD_EINVAL, "bond dimension out of [1, chi_cap]");
    need_l += dims[i];
  }
  for (int q = 0; q < si.n; ++q) need_g += 4 * (size_t)dims[q] * dims[q + 1];
  if (!finite_all(gamma, need_g) || !finite_all(lambda, need_l))
    return fail(PTEBD_EINVAL, "non-finite input");
  PT_CHECK(set_device(h));
  PT_HIP(hipStreamSynchronize(h->stream));
  std::vector<char> tmp;
  size_t go = 0, lo = 0;
  for (int q = 0; q < si.n; ++q) {
    const int cl = dims[q], cm = dims[q + 1];
    const size_t cnt = 2 * (size_t)cl * cm;
    tmp.resize(cnt * h->celem);
    for (int a = 0; a < cl; ++a)
      for (int p = 0; p < 2; ++p)
        for (int m = 0; m < cm; ++m) {
          const size_t dst = (size_t)p * cl * cm + (size_t)m * cl + a;
          const size_t src = go + 2 * (((size_t)a * 2 + p) * cm + m);
          if (h->precision == PTEBD_FP64) {
            cplx<double>& z = ((cplx<double>*)tmp.data())[dst];
            z.re = gamma[src];
            z.im = gamma[src + 1];
          } else {
            cplx<float>& z = ((cplx<float>*)tmp.data())[dst];
            z.re = (float)gamma[src];
            z.im = (float)gamma[src + 1];
          }
        }
    PT_HIP(hipMemcpy(h->gamma_slot(s, q), tmp.data(), cnt * h->celem, hipMemcpyHostToDevice));
    go += 2 * cnt;
  }
  for (int i = 0; i <= si.n; ++i) {
    PT_HIP(hipMemcpy(h->lam_slot(s, i), lambda + lo, sizeof(double) * dims[i], hipMemcpyHostToDevice));
    lo += dims[i];
  }
  for (int i = 0; i <= si.n; ++i) si.dims[i] = dims[i];
  si.prod_nu = 1.0;
  si.prod_fid = 1.0;
  return PTEBD_OK;
}

int ptebd_debug_theta(ptebd_mps_t h, int s, int q, const double* gate, double* out) {
  PT_CHECK(check_state(h, s));
  StateInfo& si = h->st[s];
  if (q < 0 || q + 1 >= si.n) return fail(PTEBD_EINVAL, "bond q out of range");
  if (!out) return fail(PTEBD_EINVAL, "null output");
  if (gate && !finite_all(gate, 32)) return fail(PTEBD_EINVAL, "non-finite gate entry");
  PT_CHECK(set_device(h));
  const int cl = si.dims[q], cm = si.dims[q + 1], cr = si.dims[q + 2];
  GateDesc d;
  std::memset(&d, 0, sizeof(d));
  d.cl = cl;
  d.cm = cm;
  d.cr = cr;
  const int m = 2 * cl, nn = 2 * cr;
  d.transposed = nn > m;
  d.R = std::max(m, nn);
  d.C = std::min(m, nn);
  d.has_gate = gate ? 1 : 0;
  d.gq = h->gamma_slot(s, q);
  d.gq1 = h->gamma_slot(s, q + 1);
  d.lam_l = h->lam_slot(s, q);
  d.lam_m = h->lam_slot(s, q + 1);
  d.lam_r = h->lam_slot(s, q + 2);
  const size_t welems = (size_t)d.R * d.C;
  PT_CHECK(h->work.ensure(welems * h->celem));
  PT_CHECK(h->desc.ensure(sizeof(GateDesc)));
  PT_CHECK(h->gates.ensure(sizeof(double) * 32));
  d.w = h->work.p;
  d.gate = gate ? (const double*)h->gates.p : nullptr;
  if (gate) PT_HIP(hipMemcpy(h->gates.p, gate, sizeof(double) * 32, hipMemcpyHostToDevice));
  PT_HIP(hipMemcpy(h->desc.p, &d, sizeof(d), hipMemcpyHostToDevice));
  const int tiles = ((cl + 31) / 32) * ((cr + 31) / 32);
  if (h->precision == PTEBD_FP64)
    ptebd::launch_theta<double>((const GateDesc*)h->desc.p, 1, tiles, h->stream);
  else
    ptebd::launch_theta<float>((const GateDesc*)h->desc.p, 1, tiles, h->stream);
  PT_HIP(hipGetLastError());
  PT_HIP(hipStreamSynchronize(h->stream));
  std::vector<char> tmp(welems * h->celem);
  PT_HIP(hipMemcpy(tmp.data(), h->work.p, tmp.size(), hipMemcpyDeviceToHost));
  // device row index s' * chi_q + a  ->  documented row index a * 2 + s'
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < nn; ++c) {
      const size_t src = d.transposed ? (size_t)r * d.R + c : (size_t)c * d.R + r;
      const int a = r % cl, sp = r / cl;
      const size_t orow = (size_t)a * 2 + sp;
      double re, im;
      if (h->precision == PTEBD_FP64) {
        const cplx<double> z = ((const cplx<double>*)tmp.data())[src];
        re = z.re;
        im = z.im;
      } else {
        const cplx<float> z = ((const cplx<float>*)tmp.data())[src];
        re = z.re;
        im = z.im;
      }
      if (d.transposed) im = -im;
      out[2 * (orow * nn + c)] = re;
      out[2 * (orow * nn + c) + 1] = im;
    }
  return PTEBD_OK;
}

}  // extern "C"

namespace {

template <class T>
int svd_batched_t(int precision, int batch, int m, int n, const double* a, double* s, double* u,
                  double* vh, int32_t* sweeps, int max_sweeps, double tol_factor,
                  hipStream_t stream) {
  const bool tr = n > m;
  const int R = std::max(m, n), C = std::min(m, n);
  const size_t wel = (size_t)R * C, vel = (size_t)C * C;
  DevBuf work, desc, outb;
  PT_CHECK(work.ensure(sizeof(cplx<T>) * (wel + vel) * batch));
  PT_CHECK(desc.ensure(sizeof(GateDesc) * batch));
  const OutLayout L = out_layout(batch, C);
  PT_CHECK(outb.ensure(L.total));
  std::vector<cplx<T>> hw(wel * batch);
  for (int b = 0; b < batch; ++b)
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) {
        const double re = a[2 * (((size_t)b * m + i) * n + j)];
        const double im = a[2 * (((size_t)b * m + i) * n + j) + 1];
        cplx<T> z;
        z.re = (T)re;
        if (!tr) {
          z.im = (T)im;
          hw[b * wel + (size_t)j * R + i] = z;
        } else {
          z.im = (T)(-im);
          hw[b * wel + (size_t)i * R + j] = z;
        }
      }
  std::vector<GateDesc> d(batch);
  for (int b = 0; b < batch; ++b) {
    std::memset(&d[b], 0, sizeof(GateDesc));
    d[b].R = R;
    d[b].C = C;
    d[b].transposed = tr;
    d[b].w = (char*)work.p + sizeof(cplx<T>) * wel * b;
    d[b].v = (char*)work.p + sizeof(cplx<T>) * (wel * batch + vel * b);
    d[b].chi_max = 0;
    d[b].stabilize = 0;
    d[b].lam_m = nullptr;
  }
  auto cleanup = [&](int code) {
    work.release();
    desc.release();
    outb.release();
    return code;
  };
  if (hipMemcpy(work.p, hw.data(), sizeof(cplx<T>) * wel * batch, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(desc.p, d.data(), sizeof(GateDesc) * batch, hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(PTEBD_EDEVICE, "upload failed"));
  const LayerOut lo = make_layer_out(outb.p, L, C);
  int32_t counter = 0;
  int n_unconv = 0;
  int st = run_jacobi<T>(nullptr, stream, (const GateDesc*)desc.p, batch, C, lo, precision,
                         max_sweeps,
                         tol_factor, 1, 0.0, 1, &counter, &n_unconv, nullptr);
  if (st < 0) return cleanup(st);
  ptebd::launch_finalize<T>((const GateDesc*)desc.p, batch, 0.0, lo, stream);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess)
    return cleanup(fail(PTEBD_EDEVICE, "svd kernels failed"));
  std::vector<double> sig((size_t)batch * C);
  std::vector<int32_t> perm((size_t)batch * C), sw(batch);
  std::vector<cplx<T>> hv(vel * batch);
  if (hipMemcpy(sig.data(), lo.sig, sizeof(double) * batch * C, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(perm.data(), lo.perm, sizeof(int32_t) * batch * C, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(sw.data(), lo.sweeps, sizeof(int32_t) * batch, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hw.data(), work.p, sizeof(cplx<T>) * wel * batch, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hv.data(), (char*)work.p + sizeof(cplx<T>) * wel * batch, sizeof(cplx<T>) * vel * batch,
                hipMemcpyDeviceToHost) != hipSuccess)
    return cleanup(fail(PTEBD_EDEVICE, "download failed"));
  for (int b = 0; b < batch; ++b) {
    for (int j = 0; j < C; ++j) {
      const double sj = sig[(size_t)b * C + j];
      const int pj = perm[(size_t)b * C + j];
      s[(size_t)b * C + j] = sj;
      const double inv = sj > 0 ? 1.0 / sj : 0.0;
      // left vectors (m rows) and right vectors (n columns of vh)
      for (int i = 0; i < m; ++i) {
        double re, im;
        if (!tr) {
          const cplx<T> z = hw[b * wel + (size_t)pj * R + i];
          re = z.re * inv;
          im = z.im * inv;
        } else {
          const cplx<T> z = hv[b * vel + (size_t)pj * C + i];
          re = z.re;
          im = z.im;
        }
        if (u) {
          u[2 * (((size_t)b * m + i) * C + j)] = re;
          u[2 * (((size_t)b * m + i) * C + j) + 1] = im;
        }
      }
      for (int i = 0; i < n; ++i) {
        double re, im;
        if (!tr) {
          const cplx<T> z = hv[b * vel + (size_t)pj * C + i];
          re = z.re;
          im = -z.im;
        } else {
          const cplx<T> z = hw[b * wel + (size_t)pj * R + i];
          re = z.re * inv;
          im = -z.im * inv;
        }
        if (vh) {
          vh[2 * (((size_t)b * C + j) * n + i)] = re;
          vh[2 * (((size_t)b * C + j) * n + i) + 1] = im;
        }
      }
    }
    if (sweeps) sweeps[b] = sw[b];
  }
  cleanup(0);
  if (n_unconv > 0) return fail(PTEBD_WNOCONV, "some SVDs reached the sweep cap");
  return PTEBD_OK;
}

}  // namespace

extern "C" int ptebd_svd_batched(int precision, int batch, int m, int n, const double* a,
                                 double* s, double* u, double* vh, int32_t* sweeps,
                                 int max_sweeps, double tol_factor, void* hip_stream) {
  if (precision == PTEBD_BF16X3)
    return fail(PTEBD_EINVAL, "PTEBD_BF16X3 is not built in this library (use PTEBD_FP32)");
  if (precision != PTEBD_FP64 && precision != PTEBD_FP32) return fail(PTEBD_EINVAL, "bad precision");
  if (batch < 1 || m < 1 || n < 1 || std::min(m, n) > 1024 || batch > 65535)
    return fail(PTEBD_EINVAL, "bad sizes (batch in [1, 65535], min(m, n) <= 1024)");
  if (!a || !s) return fail(PTEBD_EINVAL, "null input / output");
  if (max_sweeps < 1 || !(tol_factor > 0.0)) return fail(PTEBD_EINVAL, "bad sweep controls");
  if (!finite_all(a, 2 * (size_t)batch * m * n)) return fail(PTEBD_EINVAL, "non-finite input");
  if (precision == PTEBD_FP64)
    return svd_batched_t<double>(precision, batch, m, n, a, s, u, vh, sweeps, max_sweeps,
                                 tol_factor, (hipStream_t)hip_stream);
  return svd_batched_t<float>(precision, batch, m, n, a, s, u, vh, sweeps, max_sweeps, tol_factor,
                              (hipStream_t)hip_stream);
}
