// Shared host-side plumbing of the ACR library: error handling, the device
// memory pool, device buffers and the descriptors of batched operands.
#pragma once

#include <cstdlib>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
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
// The stream that the calling thread's library work is enqueued on (set by
// every entry point through StreamScope).
struct CurStream {
  static hipStream_t& get() {
    static thread_local hipStream_t s = nullptr;
    return s;
  }
};
struct StreamScope {
  hipStream_t saved;
  explicit StreamScope(hipStream_t s) : saved(CurStream::get()) { CurStream::get() = s; }
  ~StreamScope() { CurStream::get() = saved; }
};

// Device allocations.  By default hipMalloc / hipFree; acr_set_allocator
// installs caller callbacks (for instance a framework's caching allocator),
// which receive the stream the memory will be used on.
struct Allocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, void*) = nullptr;
  static Allocator& get() {
    static Allocator a;
    return a;
  }
};

// Bump allocation from one fixed device region (the allocation-free solve):
// while a thread has a Bump installed, every DBuf of that thread takes its
// memory from the region and releases nothing.  In count-only mode nothing is
// handed out for use (the caller issues no device work): only the bytes a
// call would take are counted.
struct Bump {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  bool count_only = false;
  void* take(size_t bytes) {
    const size_t need = (bytes + 255) & ~size_t(255);
    if (!count_only && off + need > cap)
      fail(ACR_ERR_INVALID_ARG, "the call needs more scratch memory than the allocation-free maximum");
    void* p = base + (count_only ? 0 : off);
    off += need;
    return p;
  }
  bool owns(const void* p) const {
    const char* c = static_cast<const char*>(p);
    return c >= base && c < base + cap;
  }
  static Bump*& cur() {
    static thread_local Bump* b = nullptr;
    return b;
  }
};

// Caching allocator.  A freed block is kept in the free list of the
// (thread, stream) that released it: work of that thread on that stream may
// still be pending or running and use the block, so it is handed out again
// only to later work of the same thread on the same stream, which the stream
// orders after it.  Blocks released after a device synchronisation (handle
// destruction) are idle and go to a list shared by every stream.  trim()
// returns the calling thread's cached blocks and the idle ones to the system.
class Pool {
 public:
  static Pool& get() {
    static Pool p;
    return p;
  }
  void* alloc(size_t bytes) {
    if (bytes == 0) return nullptr;
    if (Bump* b = Bump::cur()) return b->take(bytes);
    const size_t r = round(bytes);
    const Key key = cur_key();
    {
      std::lock_guard<std::mutex> g(mu_);
      for (const Key& k : {key, idle_key()}) {
        auto fl = free_.find(k);
        if (fl == free_.end()) continue;
        auto it = fl->second.lower_bound(r);
        if (it != fl->second.end() && it->first <= r + r / 4) {
          void* p = it->second;
          const size_t sz = it->first;
          fl->second.erase(it);
          live_[p] = Live{sz, key.second};
          return p;
        }
      }
    }
    void* p = raw_alloc(r, key.second);
    if (!p) {
      trim();
      p = raw_alloc(r, key.second);
      if (!p) fail(ACR_ERR_OOM, "device allocation of " + std::to_string(r) + " bytes failed");
    }
    std::lock_guard<std::mutex> g(mu_);
    live_[p] = Live{r, key.second};
    total_ += r;
    return p;
  }
  void release(void* p) {
    if (!p) return;
    if (Bump* b = Bump::cur())
      if (b->owns(p)) return;
    std::lock_guard<std::mutex> g(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    free_[idle() ? idle_key() : cur_key()].emplace(it->second.bytes, p);
    live_.erase(it);
  }
  // Blocks the calling thread releases inside this scope are known to be
  // idle (the device was synchronised before).
  struct IdleScope {
    IdleScope() { idle() = true; }
    ~IdleScope() { idle() = false; }
  };
  void trim();
  size_t total() const { return total_; }
  size_t live() {
    std::lock_guard<std::mutex> g(mu_);
    return live_.size();
  }
  // Return every cached block of every thread to the current source (the
  // caller synchronises the device first).
  void release_all_cached() {
    std::lock_guard<std::mutex> g(mu_);
    for (auto& fl : free_)
      for (auto& kv : fl.second) {
        raw_free(kv.second, fl.first.second);
        total_ -= kv.first;
      }
    free_.clear();
  }

 private:
  using Key = std::pair<std::thread::id, hipStream_t>;
  struct Live {
    size_t bytes;
    hipStream_t st;
  };
  static Key cur_key() { return Key(std::this_thread::get_id(), CurStream::get()); }
  static Key idle_key() { return Key(std::thread::id(), nullptr); }
  static void* raw_alloc(size_t r, hipStream_t st) {
    void* p = nullptr;
    const Allocator& A = Allocator::get();
    if (A.alloc) return A.alloc(r, st);
    if (hipMalloc(&p, r) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  static void raw_free(void* p, hipStream_t st) {
    const Allocator& A = Allocator::get();
    if (A.free) A.free(p, st);
    else (void)hipFree(p);
  }
  static size_t round(size_t b) {
    if (b <= 4096) return 4096;
    size_t g = 1;
    while (g * 16 < b) g <<= 1;           // granularity ~ b/16, power of two
    return (b + g - 1) / g * g;
  }
  std::mutex mu_;
  std::map<Key, std::multimap<size_t, void*>> free_;
  std::map<void*, Live> live_;
  size_t total_ = 0;
  static bool& idle() {
    static thread_local bool v = false;
    return v;
  }
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
    paths_.clear();
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
  // Count `n` problems planned on a named kernel path (while any class is
  // recorded); lets tests check which variants a call used.
  void hit(const char* path, long long n) {
    if (!mask_) return;
    std::lock_guard<std::mutex> g(mu_);
    paths_[path] += n;
  }
  std::map<std::string, long long>& paths() { return paths_; }
  std::mutex& mu() { return mu_; }
  std::vector<Rec>& recs() { return recs_; }
  std::vector<DBuf<int>>& owned() { return owned_; }
  std::vector<DBuf<double>>& owned_d() { return owned_d_; }

 private:
  unsigned mask_ = 0;
  std::mutex mu_;
  std::vector<Rec> recs_;
  std::map<std::string, long long> paths_;
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
    if (!P.on(cls) || Bump::cur()) return;   // the allocation-free solve records no events
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
// below is flushed, just before the launches that read it.  Each host thread
// has its own arena; it wraps around only after a device synchronisation
// (the thread may have used several streams).
class DescArena {
 public:
  static DescArena& get() {
    static thread_local DescArena a;
    return a;
  }
  // Stage `bytes` of host data; returns the device address it will have.
  void* put(const void* data, size_t bytes, hipStream_t st);
  // An external device region for the descriptors of the calling thread (the
  // allocation-free solve): host staging in ordinary host memory, no wrap
  // (exceeding `cap` is an error), count_only: nothing is copied.
  struct External {
    std::vector<char> host;
    char* dev = nullptr;
    size_t cap = 0, off = 0, pend = 0;
    bool count_only = false;
    static External*& cur() {
      static thread_local External* e = nullptr;
      return e;
    }
  };
  // Copy everything staged since the last upload (on st).
  void upload_pending(hipStream_t st) {
    if (off_ > pend_)
      ACR_HIP(hipMemcpyAsync(dev_ + pend_, host_ + pend_, off_ - pend_, hipMemcpyHostToDevice, st));
    pend_ = off_;
  }
  ~DescArena() {
    if (host_) {
      (void)hipDeviceSynchronize();
      (void)hipHostFree(host_);
      (void)hipFree(dev_);
    }
  }

 private:
  DescArena() { grow(size_t(16) << 20); }
  void grow(size_t cap) {
    if (host_) { (void)hipHostFree(host_); (void)hipFree(dev_); }
    host_ = nullptr;
    dev_ = nullptr;
    ACR_HIP(hipHostMalloc((void**)&host_, cap, hipHostMallocDefault));
    ACR_HIP(hipMalloc((void**)&dev_, cap));
    cap_ = cap;
    off_ = pend_ = 0;
  }
  char* host_ = nullptr;
  char* dev_ = nullptr;
  size_t cap_ = 0, off_ = 0, pend_ = 0;
};

// Zero fills of up to kZeroBatch byte ranges in one launch of the library's
// fill kernel (never hipMemsetAsync).
constexpr int kZeroBatch = 32;
struct ZeroArgs {
  unsigned char* p[kZeroBatch];
  unsigned long long n[kZeroBatch];
  int count;
};
void zero_bytes_now(const ZeroArgs& z, hipStream_t st);

inline void desc_upload(hipStream_t st);

// ---------------------------------------------------------- deferred queue
// Every stream operation of the library (kernel launches, fills, device
// copies) is recorded here and issued in order by flush(), after a single
// upload of the job descriptors staged meanwhile.  This turns the hundreds
// of small descriptor copies of one factorisation into a few.  flush() is
// called before any host read of device data, before memory is returned to
// the system and at the end of every entry point; ops issued by flush() keep
// stream order with everything enqueued before.  One queue per host thread,
// one stream at a time: a new stream flushes the ops of the previous one.
class Queue {
 public:
  static Queue& get() {
    static thread_local Queue q;
    return q;
  }
  void op(hipStream_t st, std::function<void()> f) {
    if (dry_) return;   // planning only: nothing reaches the device
    if (!ops_.empty() && st != st_) flush();
    st_ = st;
    last_fill_.reset();
    ops_.push_back(std::move(f));
    if (eager_ > 0) {   // the device is idle: issue at once while the host plans on
      --eager_;
      flush();
    } else if (ops_.size() >= kMaxPending) {
      flush();
    }
  }
  // After a host synchronisation the device has nothing to do: the next few
  // operations are issued as soon as they are recorded.
  void device_idle() { eager_ = kEagerAfterSync; }
  // Add a zero fill to the fill launch recorded last, if that is the last
  // pending op (same stream, room left); false otherwise.
  bool append_fill(hipStream_t st, void* p, size_t bytes) {
    if (!last_fill_ || st != st_ || ops_.empty() || last_fill_->count >= kZeroBatch) return false;
    last_fill_->p[last_fill_->count] = static_cast<unsigned char*>(p);
    last_fill_->n[last_fill_->count] = bytes;
    ++last_fill_->count;
    return true;
  }
  // The fill just recorded takes later consecutive fills, as long as it is
  // still pending (recording it may have flushed the queue).
  void set_fill(hipStream_t st, std::shared_ptr<ZeroArgs> z) {
    if (st == st_ && !ops_.empty()) last_fill_ = std::move(z);
  }
  void flush() {
    if (flushing_) return;
    flushing_ = true;
    std::vector<std::function<void()>> ops;
    ops.swap(ops_);
    last_fill_.reset();
    try {
      desc_upload(st_);
      for (auto& f : ops) f();
    } catch (...) {
      flushing_ = false;
      throw;
    }
    flushing_ = false;
  }
  // Drop recorded ops (after an error: their buffers may be gone).
  void discard() {
    ops_.clear();
    last_fill_.reset();
  }
  bool empty() const { return ops_.empty(); }
  // While dry, recorded operations are dropped (a planning pass that only
  // measures the memory a call takes).
  bool dry() const { return dry_; }
  void set_dry(bool d) { dry_ = d; }

 private:
  static constexpr size_t kMaxPending = 24;   // keeps the device fed during long host planning
  std::vector<std::function<void()>> ops_;
  std::shared_ptr<ZeroArgs> last_fill_;
  int eager_ = 0;
  static constexpr int kEagerAfterSync = 2;
  hipStream_t st_ = nullptr;
  bool flushing_ = false;
  bool dry_ = false;
};

inline void queue_flush() { Queue::get().flush(); }

// Descriptor staging of the calling thread: the external region when one is
// installed, else the thread's arena.
inline void* desc_put(const void* data, size_t bytes, hipStream_t st) {
  if (DescArena::External* e = DescArena::External::cur()) {
    const size_t need = (bytes + 255) & ~size_t(255);
    if (!e->count_only && e->off + need > e->cap)
      fail(ACR_ERR_INVALID_ARG, "the call needs more descriptor memory than the allocation-free maximum");
    if (!e->count_only) {
      if (e->host.size() < e->off + need) e->host.resize(std::max(e->off + need, 2 * e->host.size()));
      std::memcpy(e->host.data() + e->off, data, bytes);
    }
    void* d = e->dev + (e->count_only ? 0 : e->off);
    e->off += need;
    return d;
  }
  return DescArena::get().put(data, bytes, st);
}
inline void desc_upload(hipStream_t st) {
  if (DescArena::External* e = DescArena::External::cur()) {
    if (!e->count_only && e->off > e->pend)
      ACR_HIP(hipMemcpyAsync(e->dev + e->pend, e->host.data() + e->pend, e->off - e->pend, hipMemcpyHostToDevice, st));
    e->pend = e->off;
    return;
  }
  DescArena::get().upload_pending(st);
}

inline void* DescArena::put(const void* data, size_t bytes, hipStream_t st) {
  (void)st;
  const size_t need = (bytes + 255) & ~size_t(255);
  if (off_ + need > cap_) {
    Queue::get().flush();              // issues the ops reading the staged range
    ACR_HIP(hipDeviceSynchronize());   // every stream this thread used is done with the arena
    off_ = pend_ = 0;
    if (need > cap_) grow(need * 2);
  }
  std::memcpy(host_ + off_, data, bytes);
  void* d = dev_ + off_;
  off_ += need;
  return d;
}

inline void Pool::trim() {
  queue_flush();   // deferred work of this thread may still use the blocks freed below
  std::lock_guard<std::mutex> g(mu_);
  bool any = false;
  for (const Key& k : {cur_key(), idle_key()}) {
    auto fl = free_.find(k);
    if (fl != free_.end() && !fl->second.empty()) any = true;
  }
  if (!any) return;
  (void)hipDeviceSynchronize();
  for (const Key& k : {cur_key(), idle_key()}) {
    auto fl = free_.find(k);
    if (fl == free_.end()) continue;
    for (auto& kv : fl->second) {
      raw_free(kv.second, k.second);
      total_ -= kv.first;
    }
    free_.erase(fl);
  }
}


// Kernel launches (and fills) recorded by the calling thread so far.
inline long long& launch_count() {
  static thread_local long long n = 0;
  return n;
}

// Record a kernel launch (timed by the profiler when its class is selected).
template <typename... KArgs, typename... Args>
void launch(hipStream_t st, int cls, double flops, double bytes, const char* kname, void (*kern)(KArgs...),
            dim3 grid, dim3 block, size_t shmem, Args... args) {
  const Phase ph = Phase::cur();
  if (Queue::get().dry()) return;
  ++launch_count();
  Queue::get().op(st, [=]() {
    ProfScope ps(cls, st, flops, bytes, ph, kname);
    hipLaunchKernelGGL(kern, grid, block, shmem, st, args...);
    ACR_HIP(hipGetLastError());
  });
}

// Record a zero fill (consecutive fills share one launch) / a device-to-device copy.
inline void memset_async(void* p, int v, size_t bytes, hipStream_t st) {
  if (!bytes) return;
  if (v != 0) fail(ACR_ERR_INTERNAL, "memset_async supports zero fills only");
  Queue& q = Queue::get();
  if (q.dry()) return;
  if (!q.append_fill(st, p, bytes)) {
    ++launch_count();
    // the new fill holds its first range before it is recorded: recording may
    // flush the queue (and run the fill) at once, and later fills then start
    // a launch of their own
    auto z = std::make_shared<ZeroArgs>();
    z->count = 1;
    z->p[0] = static_cast<unsigned char*>(p);
    z->n[0] = bytes;
    q.op(st, [=]() { zero_bytes_now(*z, st); });
    q.set_fill(st, z);
  }
}
inline void copy_d2d_async(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (!bytes) return;
  Queue::get().op(st, [=]() { ACR_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st)); });
}
// Pinned staging of the calling thread's host reads, and the event a read
// waits on.  A copy into pinned memory is queued behind the work that
// produces the data (a copy into pageable memory would first wait on the
// host for that work), and polling the event returns as soon as the copy
// is done, where a blocking stream synchronisation also pays the host
// thread's wake-up.
struct HostRead {
  char* pin = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  static HostRead& get() {
    static thread_local HostRead h;
    return h;
  }
  ~HostRead() {
    if (pin) (void)hipHostFree(pin);
    if (ev) (void)hipEventDestroy(ev);
  }
};

// Flush, copy several device ranges to the host and wait for them (one wait).
struct HostCopy {
  void* dst;
  const void* src;
  size_t bytes;
};
inline void read_many_to_host(const std::vector<HostCopy>& cs, hipStream_t st) {
  Queue::get().flush();
  HostRead& H = HostRead::get();
  if (!H.ev) ACR_HIP(hipEventCreateWithFlags(&H.ev, hipEventDisableTiming));
  size_t total = 0;
  for (const auto& c : cs) total += (c.bytes + 15) & ~size_t(15);
  if (total > H.cap) {
    if (H.pin) (void)hipHostFree(H.pin);
    H.pin = nullptr;
    H.cap = 0;
    const size_t cap = std::max(total, size_t(1) << 16);
    ACR_HIP(hipHostMalloc((void**)&H.pin, cap, hipHostMallocDefault));
    H.cap = cap;
  }
  size_t o = 0;
  for (const auto& c : cs) {
    if (c.bytes) ACR_HIP(hipMemcpyAsync(H.pin + o, c.src, c.bytes, hipMemcpyDeviceToHost, st));
    o += (c.bytes + 15) & ~size_t(15);
  }
  ACR_HIP(hipEventRecord(H.ev, st));
  hipError_t e;
  while ((e = hipEventQuery(H.ev)) == hipErrorNotReady) {
  }
  if (e != hipSuccess) ACR_HIP(e);
  o = 0;
  for (const auto& c : cs) {
    if (c.bytes) std::memcpy(c.dst, H.pin + o, c.bytes);
    o += (c.bytes + 15) & ~size_t(15);
  }
  Queue::get().device_idle();
}
// Flush, copy device data to the host and wait for it.
inline void read_to_host(void* dst, const void* src, size_t bytes, hipStream_t st) {
  read_many_to_host({HostCopy{dst, src, bytes}}, st);
}

}  // namespace acr
