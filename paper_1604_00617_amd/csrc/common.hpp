// Shared host-side plumbing of the ACR library: error handling, the device
// memory pool, device buffers and the descriptors of batched operands.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/acr.h"

namespace acr {

// ----------------------------------------------------------------- errors
struct Error : std::runtime_error {
  acr_status code;
  Error(acr_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(acr_status c, const std::string& m) { throw Error(c, m); }

#define ACR_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      ::acr::fail(e_ == hipErrorOutOfMemory ? ACR_ERR_OOM : ACR_ERR_DEVICE,            \
                  std::string(#call) + ": " + hipGetErrorString(e_) + " (" __FILE__ ":" + \
                      std::to_string(__LINE__) + ")");                                 \
  } while (0)

#define ACR_CHECK_LAUNCH() ACR_HIP(hipGetLastError())

// Issues every deferred stream operation (see Queue below).
void queue_flush();

// ------------------------------------------------------------ memory pool
// Caching allocator: freed blocks are kept per rounded size and reused by
// later requests on the same stream order (every library call uses one
// stream, so a block released after enqueued work can be handed out to work
// enqueued later on that stream without a synchronisation).
class Pool {
 public:
  static Pool& get() {
    static Pool p;
    return p;
  }
  void* alloc(size_t bytes) {
    if (bytes == 0) return nullptr;
    size_t r = round(bytes);
    {
      std::lock_guard<std::mutex> g(mu_);
      auto it = free_.lower_bound(r);
      if (it != free_.end() && it->first <= r + r / 4) {
        void* p = it->second;
        size_t sz = it->first;
        free_.erase(it);
        live_[p] = sz;
        return p;
      }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, r);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trim();
      e = hipMalloc(&p, r);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(ACR_ERR_OOM, "hipMalloc of " + std::to_string(r) + " bytes failed");
      }
    }
    std::lock_guard<std::mutex> g(mu_);
    live_[p] = r;
    total_ += r;
    return p;
  }
  void release(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    free_.emplace(it->second, p);
    live_.erase(it);
  }
  void trim() {
    queue_flush();   // deferred work may still use the blocks freed below
    std::lock_guard<std::mutex> g(mu_);
    if (!free_.empty()) (void)hipDeviceSynchronize();
    for (auto& kv : free_) {
      (void)hipFree(kv.second);
      total_ -= kv.first;
    }
    free_.clear();
  }
  size_t total() const { return total_; }

 private:
  static size_t round(size_t b) {
    if (b <= 4096) return 4096;
    size_t g = 1;
    while (g * 16 < b) g <<= 1;           // granularity ~ b/16, power of two
    return (b + g - 1) / g * g;
  }
  std::mutex mu_;
  std::multimap<size_t, void*> free_;
  std::map<void*, size_t> live_;
  size_t total_ = 0;
};

// Owning device buffer of n elements of T (from the pool).
template <typename T>
class DBuf {
 public:
  DBuf() = default;
  explicit DBuf(size_t n) { resize(n); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { reset(); p_ = o.p_; n_ = o.n_; o.p_ = nullptr; o.n_ = 0; }
    return *this;
  }
  ~DBuf() { reset(); }
  void resize(size_t n) {
    reset();
    if (n) p_ = static_cast<T*>(Pool::get().alloc(n * sizeof(T)));
    n_ = n;
  }
  void reset() {
    if (p_) Pool::get().release(p_);
    p_ = nullptr;
    n_ = 0;
  }
  T* get() const { return p_; }
  size_t size() const { return n_; }
  size_t bytes() const { return n_ * sizeof(T); }

 private:
  T* p_ = nullptr;
  size_t n_ = 0;
};

// --------------------------------------------------------- event profiler
// Opt-in timing of every launch of selected kernel classes with HIP events
// recorded on the launch stream, plus the algorithmic flops and bytes of each
// launch (counted from its shapes).
enum KClass { KC_GEMM = 0, KC_INVERSE, KC_QR, KC_APPLYQ, KC_SVD, KC_MATVEC, KC_COPY, KC_OTHER, KC_COUNT };

// Stage label of the launches recorded by this thread (set by PhaseScope;
// static strings only) and the cyclic-reduction level it belongs to.
struct Phase {
  const char* name = "-";
  int level = -1;
  static Phase& cur() {
    static thread_local Phase p;
    return p;
  }
};
struct PhaseScope {
  Phase saved;
  PhaseScope(const char* n, int level = -2) : saved(Phase::cur()) {
    Phase::cur().name = n;
    if (level != -2) Phase::cur().level = level;
  }
  ~PhaseScope() { Phase::cur() = saved; }
};

class Profiler {
 public:
  struct Rec {
    const char* phase;
    const char* kname;
    int level;
    int cls;
    hipEvent_t a, b;
    double flops, bytes;
    const int* dev_sweeps;   // SVD: per-problem sweep counts (flops filled at read time)
    int nprob, c;
    const double* dev_flops; // per-problem flops counted on the device
  };
  static Profiler& get() {
    static Profiler p;
    return p;
  }
  bool on(int cls) const { return (mask_ >> cls) & 1u; }
  void start(unsigned mask) {
    std::lock_guard<std::mutex> g(mu_);
    for (auto& r : recs_) { pool_.push_back(r.a); pool_.push_back(r.b); }
    recs_.clear();
    owned_.clear();
    owned_d_.clear();
    mask_ = mask;
  }
  hipEvent_t event() {
    if (!pool_.empty()) { hipEvent_t e = pool_.back(); pool_.pop_back(); return e; }
    hipEvent_t e;
    ACR_HIP(hipEventCreate(&e));
    return e;
  }
  void push(const Rec& r) { std::lock_guard<std::mutex> g(mu_); recs_.push_back(r); }
  std::mutex& mu() { return mu_; }
  std::vector<Rec>& recs() { return recs_; }
  std::vector<DBuf<int>>& owned() { return owned_; }
  std::vector<DBuf<double>>& owned_d() { return owned_d_; }

 private:
  unsigned mask_ = 0;
  std::mutex mu_;
  std::vector<Rec> recs_;
  std::vector<hipEvent_t> pool_;
  std::vector<DBuf<int>> owned_;
  std::vector<DBuf<double>> owned_d_;
};

struct ProfScope {
  bool act = false;
  Profiler::Rec r{};
  hipStream_t st = nullptr;
  ProfScope(int cls, hipStream_t s, double flops, double bytes, const Phase& ph = Phase::cur(),
            const char* kname = "-") {
    Profiler& P = Profiler::get();
    if (!P.on(cls)) return;
    act = true;
    st = s;
    std::lock_guard<std::mutex> g(P.mu());
    r.phase = ph.name; r.level = ph.level; r.kname = kname;
    r.cls = cls; r.flops = flops; r.bytes = bytes; r.dev_sweeps = nullptr; r.dev_flops = nullptr;
    r.a = P.event(); r.b = P.event();
    ACR_HIP(hipEventRecord(r.a, st));
  }
  ~ProfScope() {
    if (!act) return;
    (void)hipEventRecord(r.b, st);
    Profiler::get().push(r);
  }
};

// -------------------------------------------------- batched operand views
// One operand of a batched operation over problems p = (m, c): matrix index
// m (0..nmat-1) and cluster index c (0..ncl-1).  With cc = (c >> cshift) ^ cxor
// the operand of problem p starts at
//   base + (mmul*m + moff)*sm + (cc >> 1)*sc_pair + (cc & 1)*sc_odd
// and is column-major with leading dimension ld (transposed if trans).
struct BOp {
  const void* p = nullptr;
  int ld = 1;
  int trans = 0;
  int mmul = 1, moff = 0;
  long long sm = 0;
  long long sc_pair = 0, sc_odd = 0;
  int cxor = 0;
  int cshift = 0;   // cluster used = ((c >> cshift) ^ cxor)
};

// Uniform cluster stride helper: operand of cluster c at base + c*sc.
inline BOp bop(const void* p, int ld, long long sm, long long sc = 0, int trans = 0) {
  BOp o;
  o.p = p; o.ld = ld; o.sm = sm; o.sc_pair = 2 * sc; o.sc_odd = sc; o.trans = trans;
  return o;
}
inline BOp with_map(BOp o, int mmul, int moff) { o.mmul = mmul; o.moff = moff; return o; }
inline BOp swapped(BOp o) { o.cxor = 1; return o; }
inline BOp ancestor(BOp o, int shift, int x) { o.cshift = shift; o.cxor = x; return o; }
inline BOp transposed(BOp o) { o.trans = 1; return o; }

// ------------------------------------------------------- descriptor arena
// Job descriptors of grouped launches are written to pinned host memory;
// the pending range is copied to the device in one transfer when the queue
// below is flushed, just before the launches that read it.  The arena wraps
// around only after a stream synchronisation.
class DescArena {
 public:
  static DescArena& get() {
    static DescArena a;
    return a;
  }
  // Stage `bytes` of host data; returns the device address it will have.
  void* put(const void* data, size_t bytes, hipStream_t st);
  // Copy everything staged since the last upload (on st).
  void upload_pending(hipStream_t st) {
    if (off_ > pend_)
      ACR_HIP(hipMemcpyAsync(dev_ + pend_, host_ + pend_, off_ - pend_, hipMemcpyHostToDevice, st));
    pend_ = off_;
  }

 private:
  DescArena() { grow(size_t(16) << 20); }
  void grow(size_t cap) {
    if (host_) { (void)hipHostFree(host_); (void)hipFree(dev_); }
    ACR_HIP(hipHostMalloc((void**)&host_, cap, hipHostMallocDefault));
    ACR_HIP(hipMalloc((void**)&dev_, cap));
    cap_ = cap;
    off_ = pend_ = 0;
  }
  char* host_ = nullptr;
  char* dev_ = nullptr;
  size_t cap_ = 0, off_ = 0, pend_ = 0;
};

// ---------------------------------------------------------- deferred queue
// Every stream operation of the library (kernel launches, fills, device
// copies) is recorded here and issued in order by flush(), after a single
// upload of the job descriptors staged meanwhile.  This turns the hundreds
// of small descriptor copies of one factorisation into a few.  flush() is
// called before any host read of device data, before memory is returned to
// the system and at the end of every entry point; ops issued by flush() keep
// stream order with everything enqueued before.  One stream at a time: a new
// stream flushes the ops of the previous one first.
class Queue {
 public:
  static Queue& get() {
    static Queue q;
    return q;
  }
  void op(hipStream_t st, std::function<void()> f) {
    if (!ops_.empty() && st != st_) flush();
    st_ = st;
    ops_.push_back(std::move(f));
    if (ops_.size() >= kMaxPending) flush();
  }
  void flush() {
    if (flushing_) return;
    flushing_ = true;
    std::vector<std::function<void()>> ops;
    ops.swap(ops_);
    try {
      DescArena::get().upload_pending(st_);
      for (auto& f : ops) f();
    } catch (...) {
      flushing_ = false;
      throw;
    }
    flushing_ = false;
  }
  // Drop recorded ops (after an error: their buffers may be gone).
  void discard() { ops_.clear(); }
  bool empty() const { return ops_.empty(); }

 private:
  static constexpr size_t kMaxPending = 24;   // keeps the device fed during long host planning
  std::vector<std::function<void()>> ops_;
  hipStream_t st_ = nullptr;
  bool flushing_ = false;
};

inline void queue_flush() { Queue::get().flush(); }

inline void* DescArena::put(const void* data, size_t bytes, hipStream_t st) {
  const size_t need = (bytes + 255) & ~size_t(255);
  if (off_ + need > cap_) {
    Queue::get().flush();              // issues the ops reading the staged range
    ACR_HIP(hipStreamSynchronize(st));
    off_ = pend_ = 0;
    if (need > cap_) grow(need * 2);
  }
  std::memcpy(host_ + off_, data, bytes);
  void* d = dev_ + off_;
  off_ += need;
  return d;
}

// Record a kernel launch (timed by the profiler when its class is selected).
template <typename... KArgs, typename... Args>
void launch(hipStream_t st, int cls, double flops, double bytes, const char* kname, void (*kern)(KArgs...),
            dim3 grid, dim3 block, size_t shmem, Args... args) {
  const Phase ph = Phase::cur();
  Queue::get().op(st, [=]() {
    ProfScope ps(cls, st, flops, bytes, ph, kname);
    hipLaunchKernelGGL(kern, grid, block, shmem, st, args...);
    ACR_HIP(hipGetLastError());
  });
}

// Record a byte fill / a device-to-device copy.
inline void memset_async(void* p, int v, size_t bytes, hipStream_t st) {
  if (!bytes) return;
  Queue::get().op(st, [=]() { ACR_HIP(hipMemsetAsync(p, v, bytes, st)); });
}
inline void copy_d2d_async(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (!bytes) return;
  Queue::get().op(st, [=]() { ACR_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st)); });
}
// Flush, copy device data to the host and wait for it.
inline void read_to_host(void* dst, const void* src, size_t bytes, hipStream_t st) {
  Queue::get().flush();
  if (bytes) ACR_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
  ACR_HIP(hipStreamSynchronize(st));
}

}  // namespace acr
