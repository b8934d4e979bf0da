// Shared host-side plumbing of the ACR library: error handling, the device
// memory pool, device buffers and the descriptors of batched operands.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
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

class Profiler {
 public:
  struct Rec {
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
  ProfScope(int cls, hipStream_t s, double flops, double bytes) {
    Profiler& P = Profiler::get();
    if (!P.on(cls)) return;
    act = true;
    st = s;
    std::lock_guard<std::mutex> g(P.mu());
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
// Job descriptors of grouped launches: written to pinned host memory and
// copied to a device buffer on the launch stream just before the kernel that
// reads them.  The arena is recycled only after the stream has been
// synchronised (reset() is called at those points).
class DescArena {
 public:
  static DescArena& get() {
    static DescArena a;
    return a;
  }
  // Copy `bytes` of host data into the arena and enqueue its upload on st;
  // returns the device address.
  void* put(const void* data, size_t bytes, hipStream_t st) {
    const size_t need = (bytes + 255) & ~size_t(255);
    if (off_ + need > cap_) {
      ACR_HIP(hipStreamSynchronize(st));
      off_ = 0;
      if (need > cap_) grow(need * 2);
    }
    std::memcpy(host_ + off_, data, bytes);
    ACR_HIP(hipMemcpyAsync(dev_ + off_, host_ + off_, bytes, hipMemcpyHostToDevice, st));
    void* d = dev_ + off_;
    off_ += need;
    return d;
  }
  void reset() { off_ = 0; }   // only after the stream that used it is synchronised

 private:
  DescArena() { grow(size_t(8) << 20); }
  void grow(size_t cap) {
    if (host_) { (void)hipHostFree(host_); (void)hipFree(dev_); }
    ACR_HIP(hipHostMalloc((void**)&host_, cap, hipHostMallocDefault));
    ACR_HIP(hipMalloc((void**)&dev_, cap));
    cap_ = cap;
    off_ = 0;
  }
  char* host_ = nullptr;
  char* dev_ = nullptr;
  size_t cap_ = 0, off_ = 0;
};

}  // namespace acr
