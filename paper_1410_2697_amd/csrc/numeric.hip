// Numeric multifrontal factorisation (dense fronts, Sec. 4.1, and
// HODLR-compressed fronts, Sec. 4.2), the preconditioner apply (Sec. 4.1.2,
// Sec. 4.2.2) and the GMRES driver (Sec. 3).
//
// Data flow per elimination-tree level (fronts grouped by height, so every
// child is finished before its parent):
//   1. zero the level's front buffers (dense n_hat x n_hat staging in HBM),
//   2. scatter A's lower entries into them (F_bar_p, Eq. fbar),
//   3. extend-add the children's update matrices (two launches: first and
//      second children, so no two workgroups add into one entry),
//   4. dense fronts: blocked right-looking partial Cholesky (64-wide
//      panels: LDS Cholesky of the diagonal block, MFMA panel and trailing
//      updates), the explicit inverse of L_pp by recursive doubling; the
//      trailing block left in place is U_p (Eq. update),
//   5. HODLR fronts: skeleton compression of every off-diagonal block
//      (phase 1 in LDS, phase 2 on the full-block residual), one host
//      synchronisation to read the ranks, then the SMW factorisation of F_pp
//      by a bottom-up sweep over all HODLR levels, X = F_pp^{-1} V,
//      S = V^T X and the update U_p = F_ff^HODLR - W S W^T written in place.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "hostpool.h"
#include "numeric.h"
#include "prof.h"

namespace mfh {


// Device blocks are cached for reuse instead of freed: a factorisation
// allocates and releases the same sizes every time, and hipMalloc/hipFree of
// hundreds of MB cost milliseconds and synchronise the device.  Sizes are
// rounded (4 KiB below 2 MiB, 2 MiB above); a cached block serves a request
// up to 25% smaller.  When hipMalloc fails, this device's cached blocks are
// freed and the allocation retried.  Callers release a block only after the
// work that uses it has completed.
namespace {
struct DevCache {
  std::mutex mu;
  std::multimap<size_t, std::pair<int, void*>> free;   // size -> (device, block)
};
DevCache& dev_cache() {
  static DevCache* c = new DevCache();   // lives until the process ends
  return *c;
}
size_t round_bytes(size_t b) {
  const size_t big = size_t(2) << 20;
  return b <= big ? (b + 4095) & ~size_t(4095) : (b + big - 1) & ~(big - 1);
}
void* dev_malloc(size_t& b, int dev) {
  b = round_bytes(b);
  DevCache& c = dev_cache();
  {
    std::lock_guard<std::mutex> g(c.mu);
    for (auto it = c.free.lower_bound(b); it != c.free.end() && it->first <= b + b / 4; ++it)
      if (it->second.first == dev) {
        void* p = it->second.second;
        b = it->first;
        c.free.erase(it);
        return p;
      }
  }
  void* p = nullptr;
  if (hipMalloc(&p, b) == hipSuccess) return p;
  (void)hipGetLastError();
  {
    std::lock_guard<std::mutex> g(c.mu);
    for (auto it = c.free.begin(); it != c.free.end();) {
      if (it->second.first == dev) {
        (void)hipFree(it->second.second);
        it = c.free.erase(it);
      } else {
        ++it;
      }
    }
  }
  if (hipMalloc(&p, b) == hipSuccess) return p;
  (void)hipGetLastError();
  return nullptr;
}
void dev_free(void* p, size_t b, int dev) {
  DevCache& c = dev_cache();
  std::lock_guard<std::mutex> g(c.mu);
  c.free.insert({b, {dev, p}});
}
}  // namespace

void DevBuf::release() {
  if (p) {
    dev_free(p, bytes, dev);
    if (ms) ms->sub((int64_t)bytes);
  }
  p = nullptr;
  bytes = 0;
}

void DevBuf::alloc(size_t b, MemStats* m) {
  release();
  ms = m;
  if (b == 0) b = 256;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    throw Err{MF_EHIP, "no current HIP device"};
  }
  const size_t want = b;
  p = dev_malloc(b, dev);
  if (!p) throw Err{MF_ENOMEM, "device allocation of " + std::to_string(want) + " bytes failed"};
  bytes = b;
  if (ms) ms->add((int64_t)b);
}

void DevBuf::ensure(size_t b, MemStats* m, hipStream_t st) {
  if (p && b <= bytes) return;
  if (p) HIPCHK(hipStreamSynchronize(st));
  alloc(std::max(b, bytes + bytes / 2), m);
}

void DevBuf::regrow(size_t b, MemStats* m, hipStream_t st, std::vector<std::unique_ptr<DevBuf>>& retired) {
  if (p && b <= bytes) return;
  HIPCHK(hipStreamSynchronize(st));   // no launch uses the old block or `retired` any more
  retired.clear();
  alloc(b, m);                        // releases the old block before allocating
}

void DevBuf::grow(size_t b, MemStats* m, std::vector<std::unique_ptr<DevBuf>>& retired) {
  if (p && b <= bytes) return;
  const size_t want = std::max(b, bytes + bytes / 2);
  if (p) {
    auto old = std::make_unique<DevBuf>();
    old->p = p;
    old->bytes = bytes;
    old->ms = ms;
    old->dev = dev;
    p = nullptr;
    bytes = 0;
    retired.push_back(std::move(old));
  }
  alloc(want, m);
}

void* Arena::alloc(size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (chunks.empty() || off + bytes > chunks.back()->bytes) {
    // chunks grow with use (1 MiB .. 64 MiB), so small factors hold little slack
    const size_t grow = std::min<size_t>((size_t)64 << 20, std::max<size_t>((size_t)1 << 20, (size_t)used));
    size_t cb = std::max(bytes, grow);
    chunks.push_back(std::make_unique<DevBuf>());
    chunks.back()->alloc(cb, ms);
    off = 0;
  }
  void* p = static_cast<char*>(chunks.back()->p) + off;
  off += bytes;
  used += (int64_t)bytes;
  return p;
}

namespace {

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Pinned host staging.  A copy from pageable host memory is not queued: it
// returns only once the stream has reached it, so each descriptor upload or
// rank read-back would leave the device idle while the host plans the next
// launches.  Copies to and from pinned memory are queued.  Chunks come from
// a process-wide free list; an owner gives its chunks back only once its
// streams are done with them.
class PinnedPool {
 public:
  struct Chunk {
    char* p = nullptr;
    size_t bytes = 0;
  };
  static Chunk get(size_t bytes) {
    {
      std::lock_guard<std::mutex> g(mu());
      std::vector<Chunk>& fl = list();
      for (size_t i = 0; i < fl.size(); ++i)
        if (fl[i].bytes >= bytes) {
          const Chunk c = fl[i];
          fl.erase(fl.begin() + (std::ptrdiff_t)i);
          return c;
        }
    }
    Chunk c;
    c.bytes = std::max(bytes, kMinChunk);
    void* p = nullptr;
    if (hipHostMalloc(&p, c.bytes, hipHostMallocPortable) != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Err{MF_ENOMEM, "pinned host allocation of " + std::to_string(c.bytes) + " bytes failed"};
    }
    c.p = static_cast<char*>(p);
    return c;
  }
  static void put(const Chunk& c) {
    if (!c.p) return;
    std::lock_guard<std::mutex> g(mu());
    std::vector<Chunk>& fl = list();
    size_t held = 0;
    for (const Chunk& x : fl) held += x.bytes;
    if (held + c.bytes > kMaxHeld) {
      (void)hipHostFree(c.p);
      return;
    }
    fl.push_back(c);
  }

 private:
  static constexpr size_t kMinChunk = (size_t)1 << 20, kMaxHeld = (size_t)256 << 20;
  static std::mutex& mu() {
    static std::mutex m;
    return m;
  }
  // never destroyed: chunks still listed at exit go with the process
  static std::vector<Chunk>& list() {
    static std::vector<Chunk>* l = new std::vector<Chunk>();
    return *l;
  }
};

// One pinned chunk for a function's small transfers, given back once the
// stream has finished (also when the function throws).
struct PinnedScratch {
  PinnedPool::Chunk c;
  hipStream_t st;
  PinnedScratch(size_t bytes, hipStream_t s) : c(PinnedPool::get(bytes)), st(s) {}
  PinnedScratch(const PinnedScratch&) = delete;
  PinnedScratch& operator=(const PinnedScratch&) = delete;
  ~PinnedScratch() {
    (void)hipStreamSynchronize(st);
    PinnedPool::put(c);
  }
  template <typename D>
  D* as(size_t off_bytes) { return reinterpret_cast<D*>(c.p + off_bytes); }
};

// Streams and events of finished factorizations, kept per device for the
// next ones: creating a stream costs about a tenth of a millisecond.  An
// owner returns them only after synchronising them.
class HipObjPool {
 public:
  static hipStream_t stream(int dev) {
    {
      std::lock_guard<std::mutex> g(mu());
      auto& v = streams()[dev];
      if (!v.empty()) {
        hipStream_t s = v.back();
        v.pop_back();
        return s;
      }
    }
    hipStream_t s = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return s;
  }
  static hipEvent_t event(int dev) {
    {
      std::lock_guard<std::mutex> g(mu());
      auto& v = events()[dev];
      if (!v.empty()) {
        hipEvent_t e = v.back();
        v.pop_back();
        return e;
      }
    }
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return e;
  }
  static void put(int dev, hipStream_t s) {
    if (!s) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
      // not reusable: a later owner's events would land in an open capture
      hipGraph_t gr = nullptr;
      if (cs != hipStreamCaptureStatusNone && hipStreamEndCapture(s, &gr) == hipSuccess && gr)
        (void)hipGraphDestroy(gr);
      (void)hipStreamDestroy(s);
      (void)hipGetLastError();
      return;
    }
    std::lock_guard<std::mutex> g(mu());
    if (streams()[dev].size() < kKeep) streams()[dev].push_back(s);
    else (void)hipStreamDestroy(s);
  }
  static void put(int dev, hipEvent_t e) {
    if (!e) return;
    std::lock_guard<std::mutex> g(mu());
    if (events()[dev].size() < 2 * kKeep) events()[dev].push_back(e);
    else (void)hipEventDestroy(e);
  }

 private:
  static constexpr size_t kKeep = 16;
  static std::mutex& mu() {
    static std::mutex m;
    return m;
  }
  // never destroyed: what is listed at exit goes with the process
  static std::map<int, std::vector<hipStream_t>>& streams() {
    static auto* m = new std::map<int, std::vector<hipStream_t>>();
    return *m;
  }
  static std::map<int, std::vector<hipEvent_t>>& events() {
    static auto* m = new std::map<int, std::vector<hipEvent_t>>();
    return *m;
  }
};

// Uploads descriptor blobs through pinned staging.  The device copies live
// until the pool is destroyed; its owner has synchronised the streams that
// read them (and the staged copies) by then.
struct DescPool {
  Arena ar;
  std::vector<PinnedPool::Chunk> stage;
  size_t off = 0;
  DescPool() = default;
  DescPool(const DescPool&) = delete;
  DescPool& operator=(const DescPool&) = delete;
  ~DescPool() { release_staging(); }
  // the streams that copied from the staging chunks have finished
  void release_staging() {
    for (const PinnedPool::Chunk& c : stage) PinnedPool::put(c);
    stage.clear();
    off = 0;
  }
  char* upload(Blob& b, hipStream_t st) {
    if (b.h.empty()) return nullptr;
    const size_t n = b.h.size();
    void* d = ar.alloc(n);
    if (stage.empty() || off + n > stage.back().bytes) {
      stage.push_back(PinnedPool::get(n));
      off = 0;
    }
    char* h = stage.back().p + off;
    off = (off + n + 255) & ~size_t(255);
    memcpy(h, b.h.data(), n);
    b.h = std::vector<char>();
    HIPCHK(hipMemcpyAsync(d, h, n, hipMemcpyHostToDevice, st));
    return static_cast<char*>(d);
  }
  // pinned host space for n bytes of read-back, valid until the pool goes
  template <typename D>
  D* host(size_t n) {
    const size_t bytes = n * sizeof(D);
    if (stage.empty() || off + bytes > stage.back().bytes) {
      stage.push_back(PinnedPool::get(bytes));
      off = 0;
    }
    D* h = reinterpret_cast<D*>(stage.back().p + off);
    off = (off + bytes + 255) & ~size_t(255);
    return h;
  }
};

template <typename T>
GemmDesc<T> gd(const T* A, int lda, int opA, const T* B, int ldb, int opB, T* C, int ldc, int m, int n, int k,
               double alpha, double beta, int flags = 0, const int* kdev = nullptr) {
  GemmDesc<T> d{};
  d.A = A; d.B = B; d.C = C; d.kdev = kdev;
  d.m = m; d.n = n; d.k = k;
  d.lda = lda; d.ldb = ldb; d.ldc = ldc;
  d.opA = opA; d.opB = opB;
  d.flags = flags;
  d.alpha = alpha; d.beta = beta;
  return d;
}

// Split-K policy: when a batch has too few 64 x 64 output tiles to fill the
// chip, its deep products (k >= 2 * kSplitChunk) get several workgroups
// along k, writing partial sums into `part` (capacity `cap` elements; each
// problem takes its own region), followed by a fixed-order reduction.
constexpr double kPhase2WaitSeconds = 2.0;   // a phase-2 barrier wait this long gives up (status bit 8)
constexpr int kSplitTarget = 512;   // workgroups wanted per launch (two per CU)
constexpr int kSplitTargetNarrow = 1024;   // the same for right-hand-side tiles (four resident per CU)
constexpr int kSplitChunk = 128;    // smallest k range of one split
constexpr size_t kSplitFactorBytes = size_t(16) << 20;
constexpr size_t kSplitPlanBytes = size_t(16) << 20;

// Scratch of the allocation-free apply (mf_apply_noalloc): one static device
// array, which each GPU the library runs on holds until the process ends.
// It takes the apply's workspace, then kSplitPlanBytes of split-K partial
// sums (as an allocated plan has, so both applies split alike), then the step
// descriptors.
static_assert(MF_APPLY_SCRATCH_BYTES > kSplitPlanBytes, "scratch smaller than its split-K part");
static __device__ __align__(256) unsigned char scratch[MF_APPLY_SCRATCH_BYTES];

// Host side of each device's scratch: its device address (hipGetSymbolAddress
// on the first call on that device, with the device current; the array's
// name is only a host stand-in) and which handle's plan, for how many
// right-hand sides, its descriptors hold now.
struct ScratchState {
  std::mutex mu;
  char* ptr = nullptr;
  uint64_t owner = 0;
  int nrhs = 0;
};
constexpr int kMaxDevices = 64;
ScratchState& scratch_state(int dev) {
  static ScratchState s[kMaxDevices];
  if (dev < 0 || dev >= kMaxDevices) throw Err{MF_ESTATE, "device index out of range"};
  return s[dev];
}
char* scratch_address(ScratchState& S) {   // S.mu held, the device current
  if (!S.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Err{MF_EHIP, std::string("scratch address lookup failed: ") + hipGetErrorString(e)};
    }
    S.ptr = static_cast<char*>(p);
  }
  return S.ptr;
}
std::atomic<uint64_t> g_handle_ids{0};

// assigns tile0/tiles_m/tiles_n/ksplit; returns total tiles; `red` receives
// the reduction descriptors of split problems (tile0 over output tiles)
template <typename T>
int finalize_gemm(std::vector<GemmDesc<T>>& v, T* part, size_t cap, std::vector<GemmDesc<T>>& red, int& rtiles,
                  int tn = kTile, int chunk_min = kSplitChunk, int target_set = 0, size_t* used_out = nullptr) {
  red.clear();
  rtiles = 0;
  int base = 0;
  for (const auto& d : v)
    if (d.m > 0 && d.n > 0) base += cdiv(d.m, kTile) * cdiv(d.n, tn);
  const int target = target_set > 0 ? target_set : tn == kTileNarrow ? kSplitTargetNarrow : kSplitTarget;
  const int want = (part && base > 0 && 2 * base <= target) ? target / base : 1;
  size_t used = 0;
  int t = 0;
  std::vector<GemmDesc<T>> out;
  out.reserve(v.size());
  for (auto& d : v) {
    if (d.m <= 0 || d.n <= 0) continue;
    d.tiles_m = cdiv(d.m, kTile);
    d.tiles_n = cdiv(d.n, tn);
    d.ksplit = 1;
    d.kchunk = 0;
    d.part = nullptr;
    if (want > 1 && !d.kdev && d.k >= 2 * chunk_min) {
      int sp = std::min(want, d.k / chunk_min);
      const int chunk = cdiv(cdiv(d.k, sp), kGemmSplitAlign) * kGemmSplitAlign;
      sp = cdiv(d.k, chunk);
      const size_t need = (size_t)sp * d.m * d.n;
      if (sp > 1 && used + need <= cap) {
        d.ksplit = sp;
        d.kchunk = chunk;
        d.part = part + used;
        used += need;
      }
    }
    d.tile0 = t;
    t += d.tiles_m * d.tiles_n * d.ksplit;
    out.push_back(d);
    if (d.ksplit > 1) {          // the reduction always walks 64 x 64 tiles
      GemmDesc<T> r = d;
      r.tiles_n = cdiv(d.n, kTile);
      r.tile0 = rtiles;
      rtiles += r.tiles_m * r.tiles_n;
      red.push_back(r);
    }
  }
  v.swap(out);
  if (used_out) *used_out = used;
  return t;
}

template <typename S, typename D>
CopyDesc<S, D> cd(const S* src, int lds, D* dst, int ldd, int rows, int cols, double alpha = 1.0, int acc = 0) {
  CopyDesc<S, D> d{};
  d.src = src; d.dst = dst; d.lds = lds; d.ldd = ldd; d.rows = rows; d.cols = cols;
  d.alpha = alpha; d.accumulate = acc;
  return d;
}

template <typename S, typename D>
int finalize_copy(std::vector<CopyDesc<S, D>>& v) {
  int t = 0;
  std::vector<CopyDesc<S, D>> out;
  for (auto& d : v) {
    if (d.rows <= 0 || d.cols <= 0) continue;
    d.tiles_r = cdiv(d.rows, kTile);
    d.tile0 = t;
    t += d.tiles_r * cdiv(d.cols, kTile);
    out.push_back(d);
  }
  v.swap(out);
  return t;
}

// Algorithmic work of one product: 2 flops per multiply-add that touches a
// structurally nonzero operand entry and a written C entry (triangular flags
// and lower-only C count exactly), bytes = operands read once + C written
// (and read when beta != 0).
template <typename T>
double gemm_flops(const GemmDesc<T>& d, int k) {
  if (d.m <= 0 || d.n <= 0 || k <= 0) return 0.0;
  const int f = d.flags;
  const bool lowc = (f & GF_LOWER_C) != 0;
  const bool af = (f & (GF_A_LOWER | GF_A_UPPER)) != 0, bf = (f & (GF_B_LOWER | GF_B_UPPER)) != 0;
  auto arange = [&](int i, int& lo, int& hi) {
    lo = 0; hi = k;
    if (f & GF_A_LOWER) hi = std::min(hi, i + 1);
    if (f & GF_A_UPPER) lo = std::max(lo, i);
  };
  auto brange = [&](int j, int& lo, int& hi) {
    lo = 0; hi = k;
    if (f & GF_B_UPPER) hi = std::min(hi, j + 1);
    if (f & GF_B_LOWER) lo = std::max(lo, j);
  };
  double t = 0.0;
  if (af && bf) {
    for (int i = 0; i < d.m; ++i)
      for (int j = 0; j < (lowc ? std::min(i + 1, d.n) : d.n); ++j) {
        int a0, a1, b0, b1;
        arange(i, a0, a1);
        brange(j, b0, b1);
        t += std::max(0, std::min(a1, b1) - std::max(a0, b0));
      }
  } else if (bf) {
    for (int j = 0; j < d.n; ++j) {
      int b0, b1;
      brange(j, b0, b1);
      t += (double)(lowc ? std::max(d.m - j, 0) : d.m) * std::max(0, b1 - b0);
    }
  } else {
    for (int i = 0; i < d.m; ++i) {
      int a0, a1;
      arange(i, a0, a1);
      t += (double)(lowc ? std::min(i + 1, d.n) : d.n) * std::max(0, a1 - a0);
    }
  }
  return 2.0 * t;
}
template <typename T>
double gemm_bytes(const GemmDesc<T>& d, int k) {
  if (d.m <= 0 || d.n <= 0) return 0.0;
  const double mn = (d.flags & GF_LOWER_C) ? 0.5 * d.m * (d.n + 1.0) : (double)d.m * d.n;
  return sizeof(T) * ((double)d.m * k + (double)k * d.n + mn * (d.beta != 0.0 ? 2.0 : 1.0));
}

// a batch of GEMMs / copies recorded for a later upload
template <typename T>
struct GemmBatch {
  std::vector<GemmDesc<T>> v, red;
  size_t off = 0, roff = 0;
  int tiles = 0, n = 0, rtiles = 0, rn = 0;
  int tn = kTile;                            // output tile width: kTileNarrow when every n <= 16
  size_t pused = 0;                          // elements of the partial-sum area this batch writes
  std::vector<FoldDesc<T>> fdesc;            // with nfold: B sources of each descriptor (at foff)
  size_t foff = 0;
  bool nfold = false;
  double flops = 0, bytes = 0, rbytes = 0;   // work of the descriptors with a host-known k
  mutable int pid = -1;                      // timing record of the last launch
  // split: split-K partial-sum area (reused by every batch of a stream)
  void stage(Blob& b, const DevBuf* split = nullptr) {
    stage(b, split ? static_cast<T*>(split->p) : nullptr, split ? split->bytes / sizeof(T) : 0);
  }
  void stage(Blob& b, T* part, size_t cap, int chunk_min = kSplitChunk, int target = 0) {
    tn = kTileNarrow;
    for (const auto& d : v)
      if (d.n > kTileNarrow) tn = kTile;
    tiles = finalize_gemm(v, part, cap, red, rtiles, tn, chunk_min, target, &pused);
    n = (int)v.size();
    off = b.add(v);
    flops = bytes = 0;
    for (const auto& d : v)
      if (!d.kdev) {
        flops += gemm_flops(d, d.k);
        bytes += gemm_bytes(d, d.k);
      }
    stage_reductions(b);
  }
  void stage_reductions(Blob& b) {
    rn = (int)red.size();
    rtiles = 0;
    rbytes = 0;
    for (auto& d : red) {
      d.tile0 = rtiles;
      rtiles += d.tiles_m * d.tiles_n;
      rbytes += sizeof(T) * ((double)d.m * d.n * (d.ksplit + (d.beta != 0.0 ? 2 : 1)));
    }
    if (rn) roff = b.add(red);
  }
  // After this batch is staged: each descriptor whose B is in `foldable`
  // (an output of the staged batch p that nothing reads afterwards) takes
  // the partial slices of the split products of p that write it as its B
  // sources.  The C arrays so folded are appended to `folded`; a descriptor
  // whose B does not line up with p's outputs reads B as usual.
  void resolve_folds(const GemmBatch& p, const std::unordered_set<const T*>& foldable, Blob& b,
                     std::vector<const T*>& folded) {
    nfold = false;
    if (tn != kTileNarrow || foldable.empty()) return;   // only the 64 x 16 tile kernel folds
    std::unordered_map<const T*, const GemmDesc<T>*> out;
    for (const auto& q : p.v) out.emplace(q.C, &q);
    auto find = [&](const T* c) -> const GemmDesc<T>* {
      auto it = out.find(c);
      return it == out.end() ? nullptr : it->second;
    };
    auto fits = [&](const GemmDesc<T>* q, const GemmDesc<T>& d) {
      return q && q->ldc == d.ldb && q->n == d.n && !(q->flags & GF_LOWER_C) && q->ksplit <= kFoldSlices;
    };
    fdesc.assign(v.size(), FoldDesc<T>{});
    for (size_t i = 0; i < v.size(); ++i) {
      const GemmDesc<T>& d = v[i];
      if (!foldable.count(d.B) || d.opB != 0 || d.arow || d.brow || d.kdev ||
          (d.flags & (GF_B_LOWER | GF_B_UPPER | GF_B_BF16)))
        continue;
      const GemmDesc<T>* src[2] = {find(d.B), nullptr};
      if (!fits(src[0], d) || src[0]->m > d.k) continue;
      if (src[0]->m < d.k) {
        src[1] = find(d.B + src[0]->m);
        if (!fits(src[1], d) || src[0]->m + src[1]->m != d.k) continue;
      }
      FoldDesc<T>& f = fdesc[i];
      f.split = src[0]->m;
      for (int s = 0; s < 2; ++s) {
        if (!src[s] || src[s]->ksplit <= 1) continue;
        f.part[s] = src[s]->part;
        f.slices[s] = src[s]->ksplit;
        f.ld[s] = src[s]->m;
        f.alpha[s] = src[s]->alpha;
        f.beta[s] = src[s]->beta;
        nfold = true;
        folded.push_back(src[s]->C);
      }
    }
    if (nfold) foff = b.add(fdesc);
    else fdesc.clear();
  }
  // After resolve_folds: the reductions of the folded outputs are left out.
  void drop_reductions(Blob& b, const std::vector<const T*>& folded) {
    if (folded.empty() || red.empty()) return;
    const std::unordered_set<const T*> gone(folded.begin(), folded.end());
    std::vector<GemmDesc<T>> keep;
    for (const auto& d : red)
      if (!gone.count(d.C)) keep.push_back(d);
    if (keep.size() == red.size()) return;
    red.swap(keep);
    stage_reductions(b);
  }
  void launch(const char* base, hipStream_t st) const {
    if (n && nfold) {
      pid = prof_begin(pk<T>(PK_GEMMNF_F64), st, flops, bytes);
      launch_gemm_fold<T>(reinterpret_cast<const GemmDesc<T>*>(base + off),
                          reinterpret_cast<const FoldDesc<T>*>(base + foff), n, tiles, st);
      prof_end(pid, st);
    } else if (n) {
      pid = prof_begin(pk<T>(tn == kTileNarrow ? PK_GEMMN_F64 : PK_GEMM_F64), st, flops, bytes);
      launch_gemm<T>(reinterpret_cast<const GemmDesc<T>*>(base + off), n, tiles, st, tn);
      prof_end(pid, st);
    }
    if (rn) {
      const int q = prof_begin(pk<T>(PK_GEMM_REDUCE_F64), st, 0.0, rbytes);
      launch_gemm_reduce<T>(reinterpret_cast<const GemmDesc<T>*>(base + roff), rn, rtiles, st);
      prof_end(q, st);
    }
  }
};
template <typename S, typename D>
struct CopyBatch {
  std::vector<CopyDesc<S, D>> v;
  size_t off = 0;
  int tiles = 0, n = 0;
  void stage(Blob& b) { tiles = finalize_copy(v); n = (int)v.size(); off = b.add(v); }
  void launch(const char* base, hipStream_t st) const {
    if (n) launch_copy<S, D>(reinterpret_cast<const CopyDesc<S, D>*>(base + off), n, tiles, st);
  }
};

template <typename T>
void potrf_work(const std::vector<PotrfDesc<T>>& v, double& flops, double& bytes) {
  flops = bytes = 0;
  for (const auto& d : v) {
    const double n = d.n;
    flops += n * n * n / 3.0 * (d.Inv ? 2.0 : 1.0);
    bytes += sizeof(T) * (n * (n + 1) * (d.Inv ? 1.5 : 1.0));
  }
}
template <typename T>
void timed_potrf(const PotrfDesc<T>* d, const std::vector<PotrfDesc<T>>& hv, int nmax, int* status, hipStream_t st) {
  double fl, by;
  potrf_work(hv, fl, by);
  const int id = prof_begin(pk<T>(nmax <= 64 ? PK_POTRF64_F64 : PK_POTRF128_F64), st, fl, by);
  launch_potrf<T>(d, (int)hv.size(), nmax, status, st);
  prof_end(id, st);
}

}  // namespace

int64_t workspace_plan(const Symbolic& s, std::vector<int64_t>& reg_off, std::vector<int64_t>& reg_elems,
                       std::vector<int64_t>& front_elem_off, const std::vector<char>* staged) {
  const int H = (int)s.levels.size();
  reg_off.assign(H, 0);
  reg_elems.assign(H, 0);
  front_elem_off.assign(s.fronts.size(), 0);
  struct Iv { int64_t off, len; int end; };
  std::vector<Iv> live;
  int64_t peak = 0;
  for (int h = 0; h < H; ++h) {
    int64_t tot = 0;
    int end = h;
    for (int p : s.levels[h]) {
      front_elem_off[p] = tot;
      if (staged && !(*staged)[p]) continue;   // never staged densely
      const int64_t nn = s.fronts[p].n();
      tot += (nn * nn + 63) & ~int64_t(63);
      const int par = s.fronts[p].parent;
      end = std::max(end, par >= 0 ? s.fronts[par].height : h);
    }
    live.erase(std::remove_if(live.begin(), live.end(), [&](const Iv& v) { return v.end < h; }), live.end());
    std::sort(live.begin(), live.end(), [](const Iv& a, const Iv& b) { return a.off < b.off; });
    int64_t pos = 0;
    for (const Iv& v : live) {
      if (v.off - pos >= tot) break;
      pos = std::max(pos, v.off + v.len);
    }
    reg_off[h] = pos;
    reg_elems[h] = tot;
    live.push_back({pos, tot, end});
    peak = std::max(peak, pos + tot);
  }
  return peak;
}

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

std::atomic<long long> g_phase2_wait_override{0};
std::atomic<bool> g_record_block_errors{false};

// Message for the breakdown bits of the device status word.
const char* breakdown_msg(int status) {
  if (status & 1) return "non-positive pivot in a Cholesky factorisation";
  if (status & 4) return "singular SMW capacitance matrix";
  return "a block to compress holds a value that is not finite (the factorisation broke down)";
}

// Ticks of the device's constant-rate clock a phase-2 workgroup waits at a
// barrier before it gives up; a test override (set_phase2_wait_ticks) wins.
long long phase2_wait_ticks(int dev) {
  const long long o = g_phase2_wait_override.load();
  if (o != 0) return o;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) {
    (void)hipGetLastError();
    khz = 100000;   // 100 MHz, the constant clock of CDNA parts
  }
  return (long long)(kPhase2WaitSeconds * 1000.0 * khz);
}

constexpr int kNB = 64;          // dense panel width
constexpr int kLdsMax = 160 * 1024;

}  // namespace

// =========================================================== Numeric<T> ====
template <typename T>
class Numeric : public NumericBase {
 public:
  Numeric(const Symbolic& s, const double* vals, const mf_opts& o);

  void apply(int nrhs, const double* r, double* z, hipStream_t st) override;
  void apply_noalloc(int nrhs, const double* r, double* z, hipStream_t st) override;

 private:
  struct FN {
    bool dense = true;
    T* F = nullptr;           // staging buffer (transient)
    int ld = 0;
    T* Linv = nullptr;        // dense: npiv x npiv, ld npiv
    T* Lfp = nullptr;         // dense: nf x npiv, ld nf
    T* G = nullptr;           // HODLR: npiv x w (Y columns per HODLR level, X in the first r_top)
    int w = 0, r_top = 0;
    std::vector<int> col;     // c_l per pp-tree level
    T* W = nullptr;           // HODLR: nf x r_top
    std::vector<T*> nodeU, nodeV, nodeK, leafInv;   // per pp-tree node
    std::vector<int> nodeR;   // rank per pp-tree node (internal)
    // sampled extend-add: the compressed update a parent gathers from
    const FfNode* ffnodes = nullptr;   // device: F_ff^HODLR cluster tree
    T* Wt = nullptr;                    // W S (nf x r_top)
  };
  std::vector<FN> fn;
  Arena arena;
  // sampled extend-add (Sec. 4.2.1): compressed fronts are not staged.  What
  // a parent reads of a compressed child (its F_ff^HODLR tree and W S) is
  // kept per child until the parent's level has been launched.
  bool sampled = false;
  std::vector<std::vector<std::unique_ptr<DevBuf>>> keep;   // by front
  std::vector<int64_t> upd_off_;       // each front's I_p^f in d_upd
  DevBuf scrS;                         // the level's gathered samples and pp leaf blocks
  T* keep_alloc(int p, int64_t n) {
    keep[p].push_back(std::make_unique<DevBuf>());
    keep[p].back()->alloc((size_t)std::max<int64_t>(n, 1) * sizeof(T), &ms);
    return keep[p].back()->template as<T>();
  }
  // a child's update as its parent's gather or extend-add reads it
  ChildUpd<T> child_upd(int c, const int* inv) const {
    const Front& fc = sym->fronts[c];
    ChildUpd<T> u{};
    u.inv = inv;
    u.nf = fc.nf();
    if (fn[c].F) {
      u.dense = 1;
      u.F = fn[c].F; u.ld = fn[c].ld; u.npc = fc.npiv;
    } else {
      u.nodes = fn[c].ffnodes;
      u.W = fn[c].W; u.Wt = fn[c].Wt; u.rtop = fn[c].r_top;
      u.wbf = (sizeof(T) == 4 && opts.uv_bf16) ? 1 : 0;
    }
    return u;
  }
  DescPool dp;
  // n entries of a compressed basis: T, or bfloat16 (2 bytes each) when rounded
  T* base_alloc(int64_t n, bool bf16) {
    return bf16 ? reinterpret_cast<T*>(arena.alloc_n<unsigned short>(n)) : arena.alloc_n<T>(n);
  }
  DevBuf ws, scrA, scrB, d_owner, d_asmfr, d_upd, d_adest, d_alvl, d_relmap;
  // blocks replaced by a growing scratch buffer, released at the next
  // synchronisation (the level's rank read-back, the end of the factor)
  std::vector<std::unique_ptr<DevBuf>> retired;
  DevBuf split;                   // split-K partial sums of the factor's GEMM batches
  std::vector<int64_t> relmap_off;
  // second stream for the whole-block skeleton kernels, which run beside
  // the phase-1 / factor / phase-2 chain of the larger blocks of a level
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  struct LevelBdlr {              // BDLR sets of one level's HODLR blocks
    std::vector<int> I, Iptr, J, Jptr;
    std::map<int, int> first;     // front -> index of its first block in this level
  };
  struct FrontBdlr {              // BDLR sets of one front's blocks (pointers start at 0)
    std::vector<int> I, Iptr, J, Jptr;
  };
  std::vector<LevelBdlr> lvb;
  std::vector<FrontBdlr> fbd;     // by front
  std::vector<int> bd_order;      // HODLR fronts, level by level
  std::vector<int> bd_left;       // fronts of each level still to do
  std::atomic<int> bd_next{0};
  TaskGroup workers;                 // BDLR tasks on the host pool
  std::mutex mu;
  std::condition_variable cv;
  int lvb_ready = 0;
  bool worker_failed = false;
  std::atomic<bool> cancel{false};
  hipStream_t st = nullptr;
  T* wsT = nullptr;

  void dense_level(const std::vector<int>& D);
  void hodlr_level(const std::vector<int>& H, int h);

  struct Rec {
    int kind;                 // 0 gemm T, 1 copy TT, 2 vec_asm, 4 split-K reduction, 5 gemm T with folded B
    size_t off;
    int n, tiles;
    double flops = 0, bytes = 0;
    int tn = kTile;           // gemm: output tile width
    size_t off2 = 0;          // kind 5: the FoldDesc array
  };
  struct Plan {
    int nrhs = 0;
    DevBuf work, split;
    char* desc = nullptr;
    DescPool dp;
    std::vector<Rec> recs;
    T* xn = nullptr;
    int uses = 0;                    // applies with this right-hand-side count so far
    hipGraphExec_t exec = nullptr;   // the recs recorded once (apply_graph)
    bool no_graph = false;           // recording failed: launch directly
    ~Plan() {
      if (exec) (void)hipGraphExecDestroy(exec);
    }
  };
  struct Layout {                    // workspace offsets of one right-hand-side count
    int64_t tot = 0;
    std::vector<int64_t> t_off, z_off, h_off;
    std::vector<std::vector<int64_t>> q_off, l_off;
  };
  Layout plan_layout(int nrhs) const;
  template <typename Upload>
  void build_plan(Plan& pl, int nrhs, const Layout& L, T* wk, T* part, size_t cap, Upload&& upload);
  void launch_recs(const Plan& pl, hipStream_t stream);
  hipStream_t cap = nullptr;         // stream the apply graphs are recorded on
  std::map<int, std::unique_ptr<Plan>> plans;
  Plan* get_plan(int nrhs);
  std::unique_ptr<Plan> na_plan;     // host side of the plan last placed in the scratch
  bool constructed = false;
  // Declared last, so destroyed first (also when the constructor throws):
  // device blocks go back to the allocator cache only after the work that
  // may still use them has finished.
  struct SyncGuard {
    Numeric* self;
    ~SyncGuard() {
      if (!self->constructed) (void)hipStreamSynchronize(self->st);
      if (self->side) (void)hipStreamSynchronize(self->side);
      self->wait_streams();
      if (self->cap) (void)hipStreamSynchronize(self->cap);
      HipObjPool::put(self->device, self->ev_fork);
      HipObjPool::put(self->device, self->ev_join);
      HipObjPool::put(self->device, self->side);
      HipObjPool::put(self->device, self->cap);
      (void)hipGetLastError();   // the calls above report nothing to later ones
    }
  } sync_guard{this};
};

template <typename T>
Numeric<T>::Numeric(const Symbolic& s, const double* vals, const mf_opts& o) {
  const double t0 = now_s();
  sym = &s;
  opts = o;
  uid = ++g_handle_ids;
  st = static_cast<hipStream_t>(o.stream);
  arena.ms = &ms;
  dp.ar.ms = &ms;
  HIPCHK(hipGetDevice(&device));
  const int n = s.n;
  const int nfr = (int)s.fronts.size();
  const bool hodlr = o.method == MF_METHOD_HODLR;
  sampled = hodlr && o.sampled != 0;
  if (sampled && o.adaptive == 1)
    throw Err{MF_EINVAL, "sampled extend-add needs adaptive 0 or 2 (the whole-block phase reads every entry)"};
  if (!sampled && o.adaptive == 2) throw Err{MF_EINVAL, "adaptive 2 (the sampled cross) needs sampled = 1"};

  d_rowptr.alloc((n + 1) * sizeof(int), &ms);
  d_colind.alloc(s.nnz * sizeof(int), &ms);
  d_vals.alloc(s.nnz * sizeof(double), &ms);
  d_perm.alloc(n * sizeof(int), &ms);
  d_iperm.alloc(n * sizeof(int), &ms);
  d_status.alloc(sizeof(int), &ms);
  {
    // A's pattern, values and the permutation go through pinned staging
    // (filled by the host threads), so the copies are queued and the host
    // goes on planning while they run
    struct Up { void* dst; const void* src; size_t bytes; };
    const Up ups[5] = {{d_rowptr.p, s.rowptr.data(), (size_t)(n + 1) * sizeof(int)},
                       {d_colind.p, s.colind.data(), (size_t)s.nnz * sizeof(int)},
                       {d_vals.p, vals, (size_t)s.nnz * sizeof(double)},
                       {d_perm.p, s.perm.data(), (size_t)n * sizeof(int)},
                       {d_iperm.p, s.iperm.data(), (size_t)n * sizeof(int)}};
    for (const Up& u : ups) {
      char* h = dp.host<char>(u.bytes);
      const size_t ch = 1 << 20;
      const int nch = (int)((u.bytes + ch - 1) / ch);
      parallel_for(nch, 1, [&](int b, int e, int) {
        for (int c = b; c < e; ++c) {
          const size_t o = (size_t)c * ch;
          memcpy(h + o, static_cast<const char*>(u.src) + o, std::min(ch, u.bytes - o));
        }
      });
      HIPCHK(hipMemcpyAsync(u.dst, h, u.bytes, hipMemcpyHostToDevice, st));
    }
  }
  launch_fill<int>(d_status.as<int>(), 1, 0, st);

  fn.resize(nfr);
  keep.resize(nfr);
  for (int p = 0; p < nfr; ++p) {
    const Front& f = s.fronts[p];
    fn[p].dense = !hodlr || f.n() < o.n_c;
    fn[p].ld = f.n();
  }
  if (hodlr) {
    side = HipObjPool::stream(device);
    ev_fork = HipObjPool::event(device);
    ev_join = HipObjPool::event(device);
  }

  // BDLR sets are host graph work: worker threads take the HODLR fronts in
  // level order while the device factors the levels below; a level is ready
  // once all its fronts are done.
  const int H = (int)s.levels.size();
  lvb.assign(H, {});
  fbd.assign(s.fronts.size(), {});
  bd_left.assign(H, 0);
  bd_order.clear();
  for (int h = 0; h < H; ++h)
    for (int p : s.levels[h])
      if (!fn[p].dense) {
        bd_order.push_back(p);
        ++bd_left[h];
      }
  while (lvb_ready < H && bd_left[lvb_ready] == 0) ++lvb_ready;
  struct Joiner {
    Numeric* self;
    ~Joiner() {
      self->cancel = true;
      self->workers.wait();
    }
  } joiner{this};
  if (hodlr && !bd_order.empty()) {
    // at most one task per worker thread (none stays queued, where a thread
    // that helps while it waits could pick it up and be held by it), and two
    // threads' worth of CPU left to this thread and the runtime, which plan
    // and launch the levels meanwhile
    const int ntasks = std::max(1, std::min<int>(max_workers() - 3, (int)bd_order.size()));
    workers.add(ntasks);
    for (int t = 0; t < ntasks; ++t)
      HostPool::get().submit([this, H]() {
        BdlrScratch w;
        for (;;) {
          const int i = bd_next.fetch_add(1);
          if (i >= (int)bd_order.size() || cancel) {
            workers.done();
            return;
          }
          const int p = bd_order[i];
          const int h = sym->fronts[p].height;
          bool ok = true;
          try {
            FrontBdlr& f = fbd[p];
            f.Iptr.assign(1, 0);
            f.Jptr.assign(1, 0);
            bdlr_front(*sym, p, opts.bdlr_depth, opts.bdlr_cap, w, f.I, f.Iptr, f.J, f.Jptr);
          } catch (...) {
            ok = false;
          }
          std::lock_guard<std::mutex> g(mu);
          if (!ok) worker_failed = true;
          --bd_left[h];
          while (lvb_ready < H && bd_left[lvb_ready] == 0) ++lvb_ready;
          if (worker_failed) lvb_ready = H;
          cv.notify_all();
        }
      });
  }
  // ---- front workspace plan: one region per level, first fit over offsets
  std::vector<int64_t> reg_off(H), reg_elems(H);
  std::vector<int64_t> front_elem_off(nfr);
  {
    std::vector<char> staged(nfr, 1);
    if (sampled)
      for (int p = 0; p < nfr; ++p) staged[p] = fn[p].dense;   // compressed fronts: samples only
    const int64_t peak = workspace_plan(s, reg_off, reg_elems, front_elem_off, &staged);
    ws.alloc(std::max<int64_t>(peak, 1) * sizeof(T), &ms);
    split.alloc(kSplitFactorBytes, &ms);
    info.workspace_bytes = peak * (int64_t)sizeof(T);
  }
  wsT = ws.as<T>();
  for (int h = 0; h < H; ++h)
    for (int p : s.levels[h])
      fn[p].F = (sampled && !fn[p].dense) ? nullptr : wsT + reg_off[h] + front_elem_off[p];

  // ---- assembly tables (A's entries are placed level by level on the
  // device: front of each index, the fronts' buffers and update sets) and the
  // relative maps, staged through pinned memory
  {
    int* owner_h = dp.host<int>((size_t)std::max(n, 1));
    AsmFront* fr_h = dp.host<AsmFront>((size_t)std::max(nfr, 1));
    std::vector<int64_t> upd_off(nfr + 1, 0);
    relmap_off.assign(nfr, 0);
    int64_t nrm = 0;
    for (int p = 0; p < nfr; ++p) {
      const Front& f = s.fronts[p];
      // a front that is never staged reads A's entries itself (height -1: not assembled)
      const bool st_p = fn[p].F != nullptr;
      fr_h[p] = AsmFront{st_p ? (int64_t)(fn[p].F - wsT) : 0, f.start, f.npiv, fn[p].ld, st_p ? f.height : -1,
                         (int)upd_off[p], (int)f.upd.size()};
      upd_off[p + 1] = upd_off[p] + (int64_t)f.upd.size();
      relmap_off[p] = nrm;
      nrm += (int64_t)f.relmap.size();
    }
    const int64_t nupd = upd_off[nfr];
    upd_off_ = upd_off;
    int* upd_h = dp.host<int>((size_t)std::max<int64_t>(nupd, 1));
    int* relmap_h = dp.host<int>((size_t)std::max<int64_t>(nrm, 1));
    parallel_for(nfr, 64, [&](int b, int e, int) {
      for (int p = b; p < e; ++p) {
        const Front& f = s.fronts[p];
        for (int i = 0; i < f.npiv; ++i) owner_h[f.start + i] = p;
        std::copy(f.upd.begin(), f.upd.end(), upd_h + upd_off[p]);
        std::copy(f.relmap.begin(), f.relmap.end(), relmap_h + relmap_off[p]);
      }
    });
    {
      int64_t covered = 0;                  // the fronts' pivot ranges tile 0..n-1
      for (int p = 0; p < nfr; ++p) covered += s.fronts[p].npiv;
      if (covered != n) throw Err{MF_EINVAL, "symbolic analysis: fronts do not cover every index"};
    }
    d_owner.alloc((size_t)std::max(n, 1) * sizeof(int), &ms);
    d_asmfr.alloc((size_t)std::max(nfr, 1) * sizeof(AsmFront), &ms);
    d_upd.alloc((size_t)std::max<int64_t>(nupd, 1) * sizeof(int), &ms);
    d_relmap.alloc((size_t)std::max<int64_t>(nrm, 1) * sizeof(int), &ms);
    HIPCHK(hipMemcpyAsync(d_owner.p, owner_h, (size_t)n * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_asmfr.p, fr_h, (size_t)nfr * sizeof(AsmFront), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_upd.p, upd_h, (size_t)nupd * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_relmap.p, relmap_h, (size_t)nrm * sizeof(int), hipMemcpyHostToDevice, st));
    if (H > 127) throw Err{MF_EINVAL, "elimination tree deeper than 127 levels"};
    d_adest.alloc((size_t)std::max<int64_t>(s.nnz, 1) * sizeof(int64_t), &ms);
    d_alvl.alloc((size_t)std::max<int64_t>(s.nnz, 1), &ms);
    launch_asm_map(d_rowptr.as<int>(), d_colind.as<int>(), d_iperm.as<int>(), d_owner.as<int>(),
                   d_asmfr.as<AsmFront>(), d_upd.as<int>(), n, d_adest.as<int64_t>(),
                   d_alvl.as<signed char>(), st);
  }
  ranks.assign(s.nblocks, -1);

  // ---- level loop
  for (int h = 0; h < H; ++h) {
    const auto& L = s.levels[h];
    launch_fill<T>(wsT + reg_off[h], reg_elems[h], (T)0, st);
    launch_assemble<T>(wsT, d_adest.as<int64_t>(), d_alvl.as<signed char>(), d_vals.as<double>(), s.nnz, h, st);
    for (int slot = 0; slot < 2; ++slot) {
      std::vector<ExtAddDesc<T>> ev;
      std::vector<ExtAddCDesc<T>> evc;   // compressed child into a staged parent
      int tiles = 0, tiles_c = 0;
      for (int p : L) {
        const Front& f = s.fronts[p];
        if ((int)f.children.size() <= slot) continue;
        const int c = f.children[slot];
        const Front& fc = s.fronts[c];
        if (fc.nf() == 0 || !fn[p].F) continue;   // an unstaged parent gathers its children itself
        if (!fn[c].F) {
          ExtAddCDesc<T> d{};
          d.c = child_upd(c, nullptr);
          d.parent = fn[p].F; d.relmap = d_relmap.as<int>() + relmap_off[c];
          d.ldp = fn[p].ld; d.nfc = fc.nf();
          d.tiles_r = cdiv(fc.nf(), kTile);
          d.tile0 = tiles_c;
          tiles_c += d.tiles_r * d.tiles_r;
          evc.push_back(d);
          continue;
        }
        ExtAddDesc<T> d{};
        d.child = fn[c].F; d.parent = fn[p].F; d.relmap = d_relmap.as<int>() + relmap_off[c];
        d.ldc = fn[c].ld; d.npc = fc.npiv; d.nfc = fc.nf(); d.ldp = fn[p].ld;
        d.tiles_r = cdiv(fc.nf(), kTile);
        d.tile0 = tiles;
        tiles += d.tiles_r * d.tiles_r;
        ev.push_back(d);
      }
      if (!ev.empty()) {
        Blob b;
        size_t off = b.add(ev);
        char* base = dp.upload(b, st);
        double by = 0;
        for (const auto& d : ev) by += (double)d.nfc * (d.nfc + 1) / 2 * 3 * sizeof(T) + 4.0 * d.nfc;
        const int id = prof_begin(pk<T>(PK_EXTADD_F64), st, 0.0, by);
        launch_extadd<T>(reinterpret_cast<const ExtAddDesc<T>*>(base + off), (int)ev.size(), tiles, st);
        prof_end(id, st);
      }
      if (!evc.empty()) {
        Blob b;
        size_t off = b.add(evc);
        char* base = dp.upload(b, st);
        launch_extadd_c<T>(reinterpret_cast<const ExtAddCDesc<T>*>(base + off), (int)evc.size(), tiles_c, st);
      }
    }
    std::vector<int> D, Hf;
    for (int p : L) (fn[p].dense ? D : Hf).push_back(p);
    dense_level(D);
    hodlr_level(Hf, h);
    // the children's kept updates have been read by this level's launches;
    // released at the next synchronisation
    if (sampled)
      for (int p : L)
        for (int c : s.fronts[p].children) {
          for (auto& kb : keep[c]) retired.push_back(std::move(kb));
          keep[c].clear();
        }
  }
  int* hstat = dp.host<int>(1);
  HIPCHK(hipMemcpyAsync(hstat, d_status.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  const int status = *hstat;
  info.status_bits = status;
  retired.clear();
  // release transient storage (the apply has its own workspaces and descriptors)
  ws.release();
  scrA.release();
  scrB.release();
  scrS.release();
  keep.clear();
  split.release();
  d_owner.release();
  d_asmfr.release();
  d_upd.release();
  d_adest.release();
  d_alvl.release();
  dp.ar.chunks.clear();
  dp.ar.off = 0;
  dp.release_staging();
  lvb.clear();
  fbd.clear();
  info.persistent_bytes = arena.used;
  info.peak_bytes = ms.peak;
  int dn = 0, hn = 0;
  for (auto& x : fn) (x.dense ? dn : hn)++;
  info.dense_fronts = dn;
  info.hodlr_fronts = hn;
  int64_t nb = 0, rs = 0;
  int rmax = 0;
  for (int r : ranks)
    if (r >= 0) { nb++; rs += r; rmax = std::max(rmax, r); }
  info.nblocks = nb;
  info.rank_sum = rs;
  info.rank_max = rmax;
  info.factor_seconds = now_s() - t0;
  note_stream(st);
  constructed = true;
  if (status & (1 | 4 | 16)) throw Err{MF_ENOTSPD, breakdown_msg(status)};
  if (status & 2) throw Err{MF_ECAPACITY, "a block rank exceeded rank_cap"};
}

// ------------------------------------------------------------ dense fronts
template <typename T>
void Numeric<T>::dense_level(const std::vector<int>& D) {
  if (D.empty()) return;
  const Symbolic& s = *sym;
  int64_t linv_tot = 0;
  int maxnp = 0;
  for (int p : D) {
    const Front& f = s.fronts[p];
    linv_tot += (int64_t)f.npiv * f.npiv;
    maxnp = std::max(maxnp, f.npiv);
  }
  T* linv = arena.alloc_n<T>(linv_tot);
  launch_fill<T>(linv, linv_tot, (T)0, st);
  for (int p : D) {
    const Front& f = s.fronts[p];
    fn[p].Linv = linv;
    linv += (int64_t)f.npiv * f.npiv;
    if (f.nf() > 0) fn[p].Lfp = arena.alloc_n<T>((int64_t)f.nf() * f.npiv);
  }
  Blob b;
  struct Step { size_t po; int pn; std::vector<PotrfDesc<T>> pv; GemmBatch<T> panel, syrk; };
  std::vector<Step> steps;
  for (int k = 0; k < maxnp; k += kNB) {
    Step sp;
    std::vector<PotrfDesc<T>> pv;
    for (int p : D) {
      const Front& f = s.fronts[p];
      if (k >= f.npiv) continue;
      FN& x = fn[p];
      const int kb = std::min(kNB, f.npiv - k);
      const int ld = x.ld, nh = f.n();
      PotrfDesc<T> pd{};
      pd.A = x.F + k + (int64_t)k * ld; pd.lda = ld; pd.n = kb;
      pd.Inv = x.Linv + k + (int64_t)k * f.npiv; pd.ldi = f.npiv;
      pv.push_back(pd);
      const int rest = nh - k - kb;
      if (rest > 0) {
        T* P = x.F + (k + kb) + (int64_t)k * ld;
        // P <- P L_kk^{-T}   (in place: a tile owns its rows across all kb columns)
        sp.panel.v.push_back(gd<T>(P, ld, 0, pd.Inv, f.npiv, 1, P, ld, rest, kb, kb, 1.0, 0.0, GF_B_UPPER));
        // trailing lower update: T <- T - P P^T
        sp.syrk.v.push_back(gd<T>(P, ld, 0, P, ld, 1, x.F + (k + kb) + (int64_t)(k + kb) * ld, ld, rest, rest, kb,
                                  -1.0, 1.0, GF_LOWER_C));
      }
    }
    sp.pn = (int)pv.size();
    sp.po = b.add(pv);
    sp.pv = std::move(pv);
    sp.panel.stage(b, &split);
    sp.syrk.stage(b, &split);
    steps.push_back(std::move(sp));
  }
  // recursive doubling for the off-diagonal blocks of L_pp^{-1}:
  // [A 0; B C]^{-1} = [A^{-1} 0; -C^{-1} B A^{-1}  C^{-1}]
  struct Dbl { GemmBatch<T> t1, x; };
  std::vector<Dbl> dbl;
  int64_t tmax = 0;
  for (int sz = kNB; sz < maxnp; sz *= 2) {
    int64_t need = 0;
    for (int p : D) {
      const int np = s.fronts[p].npiv;
      for (int i0 = 0; i0 + sz < np; i0 += 2 * sz) need += (int64_t)std::min(sz, np - i0 - sz) * sz;
    }
    tmax = std::max(tmax, need);
  }
  scrB.grow(std::max<int64_t>(tmax, 1) * sizeof(T), &ms, retired);
  for (int sz = kNB; sz < maxnp; sz *= 2) {
    Dbl dd;
    T* tp = scrB.as<T>();
    for (int p : D) {
      const Front& f = s.fronts[p];
      const int np = f.npiv, ld = fn[p].ld;
      T* Li = fn[p].Linv;
      for (int i0 = 0; i0 + sz < np; i0 += 2 * sz) {
        const int cs = std::min(sz, np - i0 - sz);
        const T* L21 = fn[p].F + (i0 + sz) + (int64_t)i0 * ld;
        dd.t1.v.push_back(gd<T>(L21, ld, 0, Li + i0 + (int64_t)i0 * np, np, 0, tp, cs, cs, sz, sz, 1.0, 0.0,
                                GF_B_LOWER));
        dd.x.v.push_back(gd<T>(Li + (i0 + sz) + (int64_t)(i0 + sz) * np, np, 0, tp, cs, 0,
                               Li + (i0 + sz) + (int64_t)i0 * np, np, cs, sz, cs, -1.0, 0.0, GF_A_LOWER));
        tp += (int64_t)cs * sz;
      }
    }
    dd.t1.stage(b, &split);
    dd.x.stage(b, &split);
    dbl.push_back(std::move(dd));
  }
  CopyBatch<T, T> lfp;
  for (int p : D) {
    const Front& f = s.fronts[p];
    if (f.nf() > 0) lfp.v.push_back(cd<T, T>(fn[p].F + f.npiv, fn[p].ld, fn[p].Lfp, f.nf(), f.nf(), f.npiv));
  }
  lfp.stage(b);
  const char* base = dp.upload(b, st);
  int* status = d_status.as<int>();
  for (auto& sp : steps) {
    timed_potrf<T>(reinterpret_cast<const PotrfDesc<T>*>(base + sp.po), sp.pv, kNB, status, st);
    sp.panel.launch(base, st);
    sp.syrk.launch(base, st);
  }
  for (auto& dd : dbl) {
    dd.t1.launch(base, st);
    dd.x.launch(base, st);
  }
  lfp.launch(base, st);
}

// ------------------------------------------------------------ HODLR fronts
template <typename T>
void Numeric<T>::hodlr_level(const std::vector<int>& Hs, int h) {
  if (Hs.empty()) return;
  const Symbolic& s = *sym;
  const double eps = opts.eps;
  const bool adaptive = opts.adaptive == 1;   // phase 2 over the whole block
  const bool cross = opts.adaptive == 2;      // phase 2 over the sampled cross (sampled fronts)
  {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return lvb_ready > h; });
    if (worker_failed) throw Err{MF_ENOMEM, "BDLR set construction failed"};
  }
  {   // this level's sets, fronts in level order
    LevelBdlr& L = lvb[h];
    L.Iptr.assign(1, 0);
    L.Jptr.assign(1, 0);
    for (int p : Hs) {
      const FrontBdlr& f = fbd[p];
      L.first[p] = (int)L.Iptr.size() - 1;
      const int io = (int)L.I.size(), jo = (int)L.J.size();
      L.I.insert(L.I.end(), f.I.begin(), f.I.end());
      L.J.insert(L.J.end(), f.J.begin(), f.J.end());
      for (size_t k = 1; k < f.Iptr.size(); ++k) L.Iptr.push_back(io + f.Iptr[k]);
      for (size_t k = 1; k < f.Jptr.size(); ++k) L.Jptr.push_back(jo + f.Jptr[k]);
    }
  }
  const LevelBdlr& lb = lvb[h];
  const int* dI;
  const int* dJ;
  {
    Blob bb;
    const size_t oi = bb.add(lb.I), oj = bb.add(lb.J);
    const char* base = dp.upload(bb, st);
    dI = reinterpret_cast<const int*>(base + oi);
    dJ = reinterpret_cast<const int*>(base + oj);
  }
  const std::vector<int>& bIptr = lb.Iptr;
  const std::vector<int>& bJptr = lb.Jptr;
  struct BR {
    int p, bi, gb, lk, nI, nJ, kcap, capr;
    bool full;                 // whole block held in registers by one workgroup
    int nwg, wcols;            // phase 2 over nwg workgroups (0: one workgroup streams the block)
    bool slds;                 // their column slices live in LDS (else updated in place in the front)
    int *pr, *pc, *rank1, *rank;
    double* u11;
    T *M, *U, *V;
    unsigned long long* keys;
    T* cand;
  };
  const size_t coop_lds = kPhase2CoopLds, coop_lds_g = 48 * 1024;
  const int coop_capacity = phase2_coop_capacity<T>(coop_lds, true);
  const int coop_capacity_g = phase2_coop_capacity<T>(coop_lds_g, false);
  std::vector<BR> br;
  // Columns per workgroup for the slice mode: as few as spread the level's
  // multi-workgroup blocks over the resident workgroups of one launch (a
  // step's update and search then run on more compute units), never more
  // than fit a workgroup's LDS.
  int wc_target = 1;
  {
    int64_t cols = 0;
    for (int p : Hs)
      for (const Block& B : s.fronts[p].blocks) {
        const bool full = B.nr <= skreg_full_rows<T>() && B.nc <= skreg_full_cols<T>();
        if (!full && adaptive && B.nr <= kPhase2CoopMaxRows && phase2_coop_wcols<T>(B.nr) > 0) cols += B.nc;
      }
    const int64_t slots = std::max<int64_t>(1, (int64_t)coop_capacity * 7 / 8);
    wc_target = (int)std::max<int64_t>(kCoopMinCols, (cols + slots - 1) / slots);
  }
  for (int p : Hs) {
    const Front& f = s.fronts[p];
    for (int bi = 0; bi < (int)f.blocks.size(); ++bi) {
      const Block& B = f.blocks[bi];
      BR x{};
      x.p = p; x.bi = bi; x.gb = s.block_base[p] + bi; x.lk = lb.first.at(p) + bi;
      x.nI = bIptr[x.lk + 1] - bIptr[x.lk];
      x.nJ = bJptr[x.lk + 1] - bJptr[x.lk];
      x.kcap = std::min(x.nI, x.nJ);
      x.capr = std::max(std::min({B.nr, B.nc, opts.rank_cap}), x.kcap);
      x.full = B.nr <= skreg_full_rows<T>() && B.nc <= skreg_full_cols<T>();
      if (!x.full && adaptive && B.nr <= kPhase2CoopMaxRows) {
        // phase 2 over several workgroups: column slices in LDS when they fit
        // the resident workgroups, else updated in place (about 64K entries each)
        const int wc = std::min(phase2_coop_wcols<T>(B.nr), wc_target);
        const int nl = wc > 0 ? cdiv(B.nc, wc) : 0;
        if (nl > 0 && nl <= coop_capacity) {
          x.nwg = nl;
          x.wcols = cdiv(B.nc, nl);
          x.slds = true;
        } else if (phase2_coop_lds<T>(B.nr, 1, false) + 64 * sizeof(T) <= coop_lds_g) {
          int ng = std::min(coop_capacity_g, std::max(1, (int)(((int64_t)B.nr * B.nc + 65535) / 65536)));
          ng = std::min(ng, B.nc);
          x.wcols = cdiv(B.nc, std::max(ng, 1));
          x.nwg = cdiv(B.nc, x.wcols);
          while (phase2_coop_lds<T>(B.nr, x.wcols, false) > coop_lds_g) {   // keep vloc + lc within LDS
            ++x.nwg;
            x.wcols = cdiv(B.nc, x.nwg);
            x.nwg = cdiv(B.nc, x.wcols);
          }
          x.slds = false;
          if (x.nwg > coop_capacity_g) x.nwg = 0;
        }
      }
      br.push_back(x);
    }
  }
  const int nb = (int)br.size();
  // ---- compression scratch (lives until the level's last launch)
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  size_t need = al(nb * sizeof(int)) * 2 + al(nb * sizeof(double));
  int64_t nslots = 0;
  for (auto& x : br) {
    const Block& B = s.fronts[x.p].blocks[x.bi];
    if (x.nwg > 0) {
      nslots += 2 * x.nwg;
      need += al((size_t)2 * x.nwg * B.nr * sizeof(T));
    }
    need += 2 * al(std::max(x.capr, 1) * sizeof(int));
    if (!x.full) need += al((size_t)std::max(x.kcap * x.kcap, 1) * sizeof(T));
    need += al((size_t)B.nr * x.capr * sizeof(T)) + al((size_t)B.nc * x.capr * sizeof(T));
  }
  need += al((size_t)std::max<int64_t>(nslots, 1) * sizeof(unsigned long long));
  scrA.regrow(need, &ms, st, retired);
  char* cur = static_cast<char*>(scrA.p);
  auto take = [&](size_t bytes) { char* r = cur; cur += al(bytes); return r; };
  // every multi-workgroup block's tagged key slots, in one range
  unsigned long long* slots =
      reinterpret_cast<unsigned long long*>(take((size_t)std::max<int64_t>(nslots, 1) * sizeof(unsigned long long)));
  int64_t slot_off = 0;
  int* rank1 = reinterpret_cast<int*>(take(nb * sizeof(int)));
  int* rankf = reinterpret_cast<int*>(take(nb * sizeof(int)));
  double* u11 = reinterpret_cast<double*>(take(nb * sizeof(double)));
  for (int i = 0; i < nb; ++i) {
    BR& x = br[i];
    const Block& B = s.fronts[x.p].blocks[x.bi];
    x.pr = reinterpret_cast<int*>(take(std::max(x.capr, 1) * sizeof(int)));
    x.pc = reinterpret_cast<int*>(take(std::max(x.capr, 1) * sizeof(int)));
    x.M = x.full ? nullptr : reinterpret_cast<T*>(take((size_t)std::max(x.kcap * x.kcap, 1) * sizeof(T)));
    x.U = reinterpret_cast<T*>(take((size_t)B.nr * x.capr * sizeof(T)));
    x.V = reinterpret_cast<T*>(take((size_t)B.nc * x.capr * sizeof(T)));
    x.rank1 = rank1 + i;
    x.rank = rankf + i;
    x.u11 = u11 + i;
    if (x.nwg > 0) {
      x.keys = slots + slot_off;
      slot_off += 2 * x.nwg;
      x.cand = reinterpret_cast<T*>(take((size_t)2 * x.nwg * B.nr * sizeof(T)));
    }
  }
  // ---- sampled extend-add (Sec. 4.2.1): the level's fronts are never
  // assembled.  What the compression reads of a block (the whole block when
  // it fits the register kernel, else B(I,J), B(:,J) and B(I,:)) and the
  // diagonal leaf blocks of both cluster trees are gathered from A and the
  // children's updates.
  // F, ld: what the pivot kernel reads; C = B(:, J), R = B(I, :) (B_hat
  // blocks; they become the cross residuals); Il, Jl: block-local I and J
  struct Smp { const T* F; T* C; T* R; const int* I; const int* J; int ld; const int* Il; const int* Jl; };
  std::vector<Smp> smp;
  const GatherFront<T>* dgf = nullptr;   // this level's fronts for the gathers (device)
  std::map<int, int> gfi;                // front -> index in dgf
  std::map<int, std::vector<T*>> ppleaf, ffleaf;   // front -> leaf block per tree node
  if (sampled) {
    size_t tneed = 0;
    for (auto& x : br) {
      const Block& B = s.fronts[x.p].blocks[x.bi];
      tneed += x.full ? al((size_t)B.nr * B.nc * sizeof(T))
                      : al((size_t)x.nI * x.nJ * sizeof(T)) + al((size_t)B.nr * x.nJ * sizeof(T)) +
                            al((size_t)x.nI * B.nc * sizeof(T));
    }
    for (int p : Hs)
      for (const TreeNode& t : s.fronts[p].pp_tree)
        if (t.left < 0) tneed += al((size_t)t.size * t.size * sizeof(T));
    scrS.regrow(std::max<size_t>(tneed, 256), &ms, st, retired);
    char* sc = static_cast<char*>(scrS.p);
    auto stake = [&](size_t elems) { T* r = reinterpret_cast<T*>(sc); sc += al(elems * sizeof(T)); return r; };
    // index lists: block-local I and J (whole-block mode), 0, 1, 2, ... (the
    // sample buffers), and each child's map from parent positions to its update set
    std::vector<int> loc;
    std::vector<size_t> locI(nb, 0), locJ(nb, 0);
    int iota_n = 1;
    for (int i = 0; i < nb; ++i) {
      const BR& x = br[i];
      const Block& B = s.fronts[x.p].blocks[x.bi];
      if (!x.full) iota_n = std::max({iota_n, x.nI, x.nJ});
      locI[i] = loc.size();
      for (int k = bIptr[x.lk]; k < bIptr[x.lk + 1]; ++k) loc.push_back(lb.I[k] - B.r0);
      locJ[i] = loc.size();
      for (int k = bJptr[x.lk]; k < bJptr[x.lk + 1]; ++k) loc.push_back(lb.J[k] - B.c0);
    }
    const size_t iota0 = loc.size();
    for (int k = 0; k < iota_n; ++k) loc.push_back(k);
    std::vector<int> inv;
    std::map<int, size_t> inv_off;
    for (int p : Hs) {
      const Front& f = s.fronts[p];
      if (f.children.size() > 2) throw Err{MF_EINVAL, "a front with more than two children"};
      for (int c : f.children) {
        const Front& fc = s.fronts[c];
        if (fc.nf() == 0) continue;
        const size_t o = inv.size();
        inv_off[c] = o;
        inv.resize(o + f.n(), -1);
        for (int a = 0; a < fc.nf(); ++a) inv[o + fc.relmap[a]] = a;
      }
    }
    Blob bi;
    const size_t oloc = bi.add(loc), oinv = bi.add(inv);
    const char* ib = dp.upload(bi, st);
    const int* dloc = reinterpret_cast<const int*>(ib + oloc);
    const int* dinv = reinterpret_cast<const int*>(ib + oinv);
    std::vector<GatherFront<T>> gf;
    for (int p : Hs) {
      const Front& f = s.fronts[p];
      GatherFront<T> g{};
      g.start = f.start; g.npiv = f.npiv; g.nhat = f.n();
      g.upd = d_upd.as<int>() + upd_off_[p];
      for (int c : f.children)
        if (s.fronts[c].nf() > 0) g.ch[g.nchild++] = child_upd(c, dinv + inv_off.at(c));
      gfi[p] = (int)gf.size();
      gf.push_back(g);
    }
    std::vector<GatherDesc<T>> gdv;
    int64_t gtiles = 0;
    auto gat = [&](int p, const int* rows, int r0, int nr, const int* cols, int c0, int nc, T* out, int ldo) {
      if (nr <= 0 || nc <= 0) return;
      GatherDesc<T> d{};
      d.rows = rows; d.cols = cols; d.out = out;
      d.r0 = r0; d.c0 = c0; d.nr = nr; d.nc = nc; d.ldo = ldo;
      d.front = gfi.at(p);
      d.tile0 = (int)gtiles;
      gtiles += ((int64_t)nr * nc + 255) / 256;
      gdv.push_back(d);
    };
    smp.resize(nb);
    for (int i = 0; i < nb; ++i) {
      const BR& x = br[i];
      const Block& B = s.fronts[x.p].blocks[x.bi];
      if (x.full) {
        T* R = stake((size_t)B.nr * B.nc);
        gat(x.p, nullptr, B.r0, B.nr, nullptr, B.c0, B.nc, R, B.nr);
        smp[i] = Smp{R, nullptr, nullptr, dloc + locI[i], dloc + locJ[i], B.nr, dloc + locI[i], dloc + locJ[i]};
        continue;
      }
      const int* Ib = dI + bIptr[x.lk];
      const int* Jb = dJ + bJptr[x.lk];
      T* Bh = stake((size_t)x.nI * x.nJ);
      T* C = stake((size_t)B.nr * x.nJ);
      T* R = stake((size_t)x.nI * B.nc);
      gat(x.p, Ib, 0, x.nI, Jb, 0, x.nJ, Bh, std::max(x.nI, 1));
      gat(x.p, nullptr, B.r0, B.nr, Jb, 0, x.nJ, C, B.nr);
      gat(x.p, Ib, 0, x.nI, nullptr, B.c0, B.nc, R, std::max(x.nI, 1));
      smp[i] = Smp{Bh, C, R, dloc + iota0, dloc + iota0, std::max(x.nI, 1), dloc + locI[i], dloc + locJ[i]};
    }
    for (int p : Hs) {
      const Front& f = s.fronts[p];
      auto& pl = ppleaf[p];
      pl.assign(f.pp_tree.size(), nullptr);
      for (size_t k = 0; k < f.pp_tree.size(); ++k) {
        const TreeNode& t = f.pp_tree[k];
        if (t.left >= 0) continue;
        pl[k] = stake((size_t)t.size * t.size);
        gat(p, nullptr, t.off, t.size, nullptr, t.off, t.size, pl[k], t.size);
      }
      // F_ff^HODLR's leaf blocks are kept whole: they are the parent's to read
      int64_t fl_tot = 0;
      for (const TreeNode& t : f.ff_tree)
        if (t.left < 0) fl_tot += (int64_t)t.size * t.size;
      auto& fl = ffleaf[p];
      fl.assign(f.ff_tree.size(), nullptr);
      if (fl_tot == 0) continue;
      T* kp = keep_alloc(p, fl_tot);
      for (size_t k = 0; k < f.ff_tree.size(); ++k) {
        const TreeNode& t = f.ff_tree[k];
        if (t.left >= 0) continue;
        fl[k] = kp;
        kp += (int64_t)t.size * t.size;
        gat(p, nullptr, t.off, t.size, nullptr, t.off, t.size, fl[k], t.size);
      }
    }
    if (gtiles > INT32_MAX) throw Err{MF_EINVAL, "level too large for one gather launch"};
    if (!gdv.empty()) {
      Blob bg;
      const size_t ogf = bg.add(gf), ogd = bg.add(gdv);
      const char* gb = dp.upload(bg, st);
      dgf = reinterpret_cast<const GatherFront<T>*>(gb + ogf);
      launch_gather<T>(reinterpret_cast<const GatherDesc<T>*>(gb + ogd), (int)gdv.size(), (int)gtiles, dgf,
                       d_rowptr.as<int>(), d_colind.as<int>(), d_vals.as<double>(), d_perm.as<int>(), st);
    }
  }
  Blob b;
  std::vector<SkRegDesc<T>> skf, skh;
  std::vector<SkelFacDesc<T>> sf;
  std::vector<Phase2Desc<T>> p2;
  std::vector<Phase2CoopDesc<T>> p2c;
  GemmBatch<T> resid;
  int rmax1 = 1, wgs = 0, maxrc = 1;
  for (auto& x : br) {
    const Block& B = s.fronts[x.p].blocks[x.bi];
    const FN& fx = fn[x.p];
    SkRegDesc<T> d{};
    d.F = fx.F; d.ld = fx.ld; d.r0 = B.r0; d.nr = B.nr; d.c0 = B.c0; d.nc = B.nc;
    d.I = dI + bIptr[x.lk]; d.nI = x.nI;
    d.J = dJ + bJptr[x.lk]; d.nJ = x.nJ;
    const Smp* sm = sampled ? &smp[&x - br.data()] : nullptr;
    if (sm) {   // the whole block, or B_hat with I and J numbered 0, 1, ...
      d.F = sm->F; d.ld = sm->ld; d.r0 = 0; d.c0 = 0;
      d.I = sm->I; d.J = sm->J;
    }
    d.piv_r = x.pr; d.piv_c = x.pc;
    d.rank1 = x.rank1; d.rank = x.rank; d.u11 = x.u11; d.cap = x.capr;
    if (x.full) {
      d.U = x.U; d.ldu = B.nr; d.V = x.V; d.ldv = B.nc;
      skf.push_back(d);
      continue;
    }
    if (x.nI > skreg_hat_max<T>() || x.nJ > skreg_hat_max<T>())
      throw Err{MF_EINVAL, "BDLR sets larger than the pivot kernel supports: lower bdlr_cap"};
    d.M = x.M; d.ldm = std::max(x.kcap, 1);
    skh.push_back(d);
    rmax1 = std::max(rmax1, x.kcap);
    SkelFacDesc<T> f{};
    f.F = fx.F; f.ld = fx.ld; f.FR = fx.F; f.ldr = fx.ld; f.r0 = B.r0; f.nr = B.nr; f.c0 = B.c0; f.nc = B.nc;
    if (sm) {   // B(:, J) and B(I, :); pivots index the lists I and J
      f.F = sm->C; f.ld = B.nr; f.r0 = 0;
      f.FR = sm->R; f.ldr = sm->ld; f.c0 = 0;
    }
    f.piv_r = x.pr; f.piv_c = x.pc; f.M = x.M; f.ldm = std::max(x.kcap, 1); f.rank = x.rank1;
    f.U = x.U; f.ldu = B.nr; f.V = x.V; f.ldv = B.nc;
    f.wgU = cdiv(B.nr, kSkelFacRows);
    f.wg0 = wgs;
    wgs += f.wgU + cdiv(B.nc, kSkelFacRows);
    sf.push_back(f);
    if (adaptive) {
      // E = B - U V^T in place (k = phase-1 rank, read on the device)
      resid.v.push_back(gd<T>(x.U, B.nr, 0, x.V, B.nc, 1, fx.F + B.r0 + (int64_t)B.c0 * fx.ld, fx.ld, B.nr, B.nc,
                              x.kcap, -1.0, 1.0, 0, x.rank1));
      if (x.nwg > 0) {
        Phase2CoopDesc<T> q{};
        q.F = fx.F; q.ld = fx.ld; q.r0 = B.r0; q.nr = B.nr; q.c0 = B.c0; q.nc = B.nc;
        q.piv_r = x.pr; q.piv_c = x.pc; q.rank1 = x.rank1; q.u11 = x.u11;
        q.U = x.U; q.ldu = B.nr; q.V = x.V; q.ldv = B.nc; q.cap = x.capr; q.rank = x.rank;
        q.keys = x.keys; q.cand = x.cand;
        q.nwg = x.nwg; q.wcols = x.wcols;
        q.slice_lds = x.slds ? 1 : 0;
        p2c.push_back(q);
        continue;
      }
      Phase2Desc<T> q{};
      q.F = fx.F; q.ld = fx.ld; q.r0 = B.r0; q.nr = B.nr; q.c0 = B.c0; q.nc = B.nc;
      q.piv_r = x.pr; q.piv_c = x.pc; q.rank1 = x.rank1; q.u11 = x.u11;
      q.U = x.U; q.ldu = B.nr; q.V = x.V; q.ldv = B.nc; q.cap = x.capr; q.rank = x.rank;
      p2.push_back(q);
      maxrc = std::max(maxrc, B.nr + B.nc);
    }
  }
  // multi-workgroup launches: consecutive groups of blocks of one slice mode
  // whose workgroups can all be resident.  Descriptors are ordered by mode,
  // then by size, largest first: a launch lasts as long as its slowest block,
  // so blocks of like size share launches.
  std::stable_sort(p2c.begin(), p2c.end(), [](const Phase2CoopDesc<T>& a, const Phase2CoopDesc<T>& b) {
    if (a.slice_lds != b.slice_lds) return a.slice_lds > b.slice_lds;
    return (int64_t)a.nr * a.nc > (int64_t)b.nr * b.nc;
  });
  struct CoopGroup { size_t first; int n, wgs; bool slds; };
  std::vector<CoopGroup> cgroups;
  for (size_t i = 0; i < p2c.size(); ++i) {
    const bool sl = p2c[i].slice_lds != 0;
    const int capg = sl ? coop_capacity : coop_capacity_g;
    if (cgroups.empty() || cgroups.back().slds != sl || cgroups.back().wgs + p2c[i].nwg > capg)
      cgroups.push_back({i, 0, 0, sl});
    CoopGroup& g = cgroups.back();
    p2c[i].wg0 = g.wgs;
    g.wgs += p2c[i].nwg;
    ++g.n;
  }
  if (skelfac_lds<T>(rmax1) > (size_t)kLdsMax)
    throw Err{MF_EINVAL, "phase-1 rank bound too large for LDS: lower bdlr_cap"};
  if (maxrc > kLdsMax) throw Err{MF_EINVAL, "block too large for the phase-2 kernel"};
  const size_t okf = b.add(skf), okh = b.add(skh), osf = b.add(sf), op2 = b.add(p2), op2c = b.add(p2c);
  resid.stage(b, &split);
  const char* base = dp.upload(b, st);
  int* dstat = d_status.as<int>();
  // test hook: every block in float64 before compression changes the front
  const bool rec = g_record_block_errors.load() && !sampled;
  DevBuf dbgB;
  std::vector<int64_t> dbg_off(nb, 0);
  if (rec) {
    int64_t tot = 0;
    for (int i = 0; i < nb; ++i) {
      const Block& B = s.fronts[br[i].p].blocks[br[i].bi];
      dbg_off[i] = tot;
      tot += (int64_t)B.nr * B.nc;
    }
    dbgB.alloc((size_t)std::max<int64_t>(tot, 1) * sizeof(double), &ms);
    CopyBatch<T, double> cb;
    for (int i = 0; i < nb; ++i) {
      const Block& B = s.fronts[br[i].p].blocks[br[i].bi];
      const FN& fx = fn[br[i].p];
      cb.v.push_back(cd<T, double>(fx.F + B.r0 + (int64_t)B.c0 * fx.ld, fx.ld, dbgB.as<double>() + dbg_off[i], B.nr,
                                   B.nr, B.nc));
    }
    Blob bd;
    cb.stage(bd);
    const char* bdb = dp.upload(bd, st);
    cb.launch(bdb, st);
  }
  // timing records; their work is added once the ranks are back on the host
  // whole-block blocks on the side stream while the larger blocks' chain
  // runs here; joined before the ranks are read back
  const bool fork = side && !skf.empty() && !skh.empty();
  hipStream_t fst = fork ? side : st;
  if (fork) {
    HIPCHK(hipEventRecord(ev_fork, st));
    HIPCHK(hipStreamWaitEvent(side, ev_fork, 0));
  }
  const int id_f = skf.empty() ? -1 : prof_begin(pk<T>(PK_SKREG_FULL_F64), fst, 0.0, 0.0);
  launch_skreg_full<T>(reinterpret_cast<const SkRegDesc<T>*>(base + okf), (int)skf.size(), eps, opts.adaptive,
                       dstat, fst);
  prof_end(id_f, fst);
  if (fork) HIPCHK(hipEventRecord(ev_join, side));
  const int id_h = skh.empty() ? -1 : prof_begin(pk<T>(PK_SKREG_HAT_F64), st, 0.0, 0.0);
  launch_skreg_hat<T>(reinterpret_cast<const SkRegDesc<T>*>(base + okh), (int)skh.size(), eps, dstat, st);
  prof_end(id_h, st);
  const int id_s = sf.empty() ? -1 : prof_begin(pk<T>(PK_SKELFAC_F64), st, 0.0, 0.0);
  launch_skelfac<T>(reinterpret_cast<const SkelFacDesc<T>*>(base + osf), (int)sf.size(), wgs, rmax1, st);
  prof_end(id_s, st);
  int id_2 = -1;
  bool fork_joined = false;
  std::vector<int> coop_ids;
  if (cross) {
    // phase 2 on the sampled cross of every B_hat block: the samples become
    // the residuals E(:, J) = B(:, J) - U V(J, :)^T and E(I, :) =
    // B(I, :) - U(I, :) V^T (k = phase-1 rank, read on the device), then one
    // workgroup per block pivots on them
    GemmBatch<T> xres;
    std::vector<CrossDesc<T>> xd;
    int maxrc = 1;
    for (int i = 0; i < nb; ++i) {
      const BR& x = br[i];
      if (x.full) continue;
      const Block& B = s.fronts[x.p].blocks[x.bi];
      const Smp& m = smp[i];
      if (x.nJ > 0) {
        auto g = gd<T>(x.U, B.nr, 0, x.V, B.nc, 1, m.C, B.nr, B.nr, x.nJ, x.kcap, -1.0, 1.0, 0, x.rank1);
        g.brow = m.Jl;
        xres.v.push_back(g);
      }
      if (x.nI > 0) {
        auto g = gd<T>(x.U, B.nr, 0, x.V, B.nc, 1, m.R, x.nI, x.nI, B.nc, x.kcap, -1.0, 1.0, 0, x.rank1);
        g.arow = m.Il;
        xres.v.push_back(g);
      }
      CrossDesc<T> c{};
      c.EJ = m.C; c.EI = m.R; c.Il = m.Il; c.Jl = m.Jl;
      c.piv_r = x.pr; c.piv_c = x.pc; c.rank1 = x.rank1; c.u11 = x.u11;
      c.U = x.U; c.V = x.V; c.rank = x.rank; c.front = dgf + gfi.at(x.p);
      c.r0 = B.r0; c.c0 = B.c0; c.nr = B.nr; c.nc = B.nc; c.nI = x.nI; c.nJ = x.nJ; c.cap = x.capr;
      xd.push_back(c);
      maxrc = std::max(maxrc, B.nr + B.nc);
    }
    if (!xd.empty()) {
      if (maxrc > kLdsMax) throw Err{MF_EINVAL, "block too large for the cross kernel"};
      Blob bx;
      const size_t ox = bx.add(xd);
      xres.stage(bx, &split);
      const char* bxb = dp.upload(bx, st);
      xres.launch(bxb, st);
      launch_cross<T>(reinterpret_cast<const CrossDesc<T>*>(bxb + ox), (int)xd.size(), maxrc, eps,
                      d_rowptr.as<int>(), d_colind.as<int>(), d_vals.as<double>(), d_perm.as<int>(), dstat, st);
    }
  }
  if (adaptive) {
    resid.launch(base, st);
    id_2 = p2.empty() ? -1 : prof_begin(pk<T>(PK_PHASE2_F64), st, 0.0, 0.0);
    launch_phase2<T>(reinterpret_cast<const Phase2Desc<T>*>(base + op2), (int)p2.size(), maxrc, eps, dstat, st);
    prof_end(id_2, st);
    if (!p2c.empty()) {
      // The multi-workgroup launches need all their workgroups resident at
      // once: the side stream's whole-block kernels (1024-thread, register
      // heavy) finish before them rather than compete for compute units.
      if (fork) {
        HIPCHK(hipStreamWaitEvent(st, ev_join, 0));
        fork_joined = true;
      }
      const long long wait_ticks = phase2_wait_ticks(device);
      launch_fill<unsigned long long>(slots, nslots, 1ull << 63, st);   // no slot carries step 0's tag
      const auto* dc = reinterpret_cast<const Phase2CoopDesc<T>*>(base + op2c);
      for (const CoopGroup& g : cgroups) {
        const int id = prof_begin(pk<T>(g.slds ? PK_PHASE2CL_F64 : PK_PHASE2CG_F64), st, 0.0, 0.0);
        coop_ids.push_back(id);
        const hipError_t e = launch_phase2_coop<T>(dc + g.first, g.n, g.wgs, g.slds ? coop_lds : coop_lds_g, g.slds,
                                                   eps, dstat, wait_ticks, st);
        prof_end(id, st);
        if (e != hipSuccess) throw Err{MF_EHIP, std::string("phase-2 launch: ") + hipGetErrorString(e)};
      }
    }
  }
  if (fork && !fork_joined) HIPCHK(hipStreamWaitEvent(st, ev_join, 0));
  // ---- the one synchronisation of the level: ranks to the host (pinned)
  int* hb = dp.host<int>(2 * (size_t)nb + 1);
  int* hb_dev = nullptr;
  HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&hb_dev), hb, 0));
  launch_readback(rankf, nb, rank1, nb, d_status.as<int>(), hb_dev, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  const std::vector<int> hr(hb, hb + nb), h1(hb + nb, hb + 2 * nb);
  const int status = hb[2 * nb];
  retired.clear();
  if (status & 2) throw Err{MF_ECAPACITY, "a block rank exceeded rank_cap"};
  if (status & 8) throw Err{MF_EHIP, kPhase2WaitMsg};
  // a breakdown below this level (non-positive pivot, singular capacitance,
  // non-finite block entries) ends the factorisation here: what the levels
  // above would compute from it is meaningless
  if (status & (1 | 4 | 16)) throw Err{MF_ENOTSPD, breakdown_msg(status)};
  for (int i = 0; i < nb; ++i) ranks[br[i].gb] = hr[i];
  // work of the rank-dependent launches: pivot step k of complete pivoting
  // updates the active (rows - k) x (cols - k) part of its block (whole block,
  // B_hat, or the phase-2 residual); the phase-1 kernel on B_hat reads it once;
  // the factor kernel solves with the r x r LU for every row and column;
  // phase 2 makes one pass (read + write) per step plus the final search.
  auto active = [](double nr, double nc, double k0, double k1) {   // sum over k in [k0, k1) of 2 (nr-k)(nc-k)
    auto s = [&](double k) { return nr * nc * k - (nr + nc) * k * (k - 1) / 2 + (k - 1) * k * (2 * k - 1) / 6; };
    return k1 > k0 ? 2.0 * (s(k1) - s(k0)) : 0.0;
  };
  {
    double ff = 0, fb = 0, hf = 0, hb = 0, sfl = 0, sb = 0, rf = 0, rb = 0, pf = 0, pb = 0, cf = 0, cbytes = 0;
    for (int i = 0; i < nb; ++i) {
      const BR& x = br[i];
      const Block& B = s.fronts[x.p].blocks[x.bi];
      const double e = (double)B.nr * B.nc;
      if (x.full) {
        ff += active(B.nr, B.nc, 0, hr[i]);
        fb += sizeof(T) * (e + (double)(B.nr + B.nc) * hr[i]);
        continue;
      }
      const double eh = (double)x.nI * x.nJ, r1 = h1[i];
      hf += active(x.nI, x.nJ, 0, r1);
      hb += sizeof(T) * (eh + r1 * r1) + 8.0 * r1;
      sfl += (double)(B.nr + B.nc) * r1 * r1;
      sb += sizeof(T) * ((double)(B.nr + B.nc) * r1 * 2);
      if (adaptive) {
        rf += 2.0 * e * r1;
        rb += sizeof(T) * ((double)(B.nr + B.nc) * r1 + 2.0 * e);
        const double steps = hr[i] - h1[i] + 1;
        if (x.nwg > 0) {   // slices read once; per step one U and V column
          cf += active(B.nr, B.nc, r1, hr[i] + 1);
          cbytes += sizeof(T) * (e + (double)(B.nr + B.nc) * (steps - 1));
        } else {
          pf += active(B.nr, B.nc, r1, hr[i] + 1);
          pb += sizeof(T) * 2.0 * e * steps;
        }
      }
    }
    prof_add(id_f, ff, fb);
    prof_add(id_h, hf, hb);
    prof_add(id_s, sfl, sb);
    prof_add(resid.pid, rf, rb);
    prof_add(id_2, pf, pb);
    // the multi-workgroup launches share the level's work in proportion to their workgroups
    if (!coop_ids.empty()) {
      double tw = 0;
      for (const CoopGroup& g : cgroups) tw += g.wgs;
      for (size_t k = 0; k < cgroups.size(); ++k)
        prof_add(coop_ids[k], cf * cgroups[k].wgs / tw, cbytes * cgroups[k].wgs / tw);
    }
  }

  if (rec) {   // max|B| and max|B - U V^T| in float64, with the bases as computed (before any rounding)
    int64_t uv = 0;
    for (int i = 0; i < nb; ++i) {
      const Block& B = s.fronts[br[i].p].blocks[br[i].bi];
      uv += (int64_t)(B.nr + B.nc) * hr[i];
    }
    DevBuf dUV, dmax;
    dUV.alloc((size_t)std::max<int64_t>(uv, 1) * sizeof(double), &ms);
    dmax.alloc((size_t)2 * nb * sizeof(double), &ms);
    CopyBatch<T, double> cu;
    GemmBatch<double> ge;
    std::vector<MaxAbsDesc> md;
    double* up = dUV.as<double>();
    for (int i = 0; i < nb; ++i) {
      const Block& B = s.fronts[br[i].p].blocks[br[i].bi];
      double* bd = dbgB.as<double>() + dbg_off[i];
      md.push_back(MaxAbsDesc{bd, B.nr, B.nc, B.nr, 0});
      const int r = hr[i];
      if (r == 0) continue;
      cu.v.push_back(cd<T, double>(br[i].U, B.nr, up, B.nr, B.nr, r));
      cu.v.push_back(cd<T, double>(br[i].V, B.nc, up + (int64_t)B.nr * r, B.nc, B.nc, r));
      ge.v.push_back(gd<double>(up, B.nr, 0, up + (int64_t)B.nr * r, B.nc, 1, bd, B.nr, B.nr, B.nc, r, -1.0, 1.0));
      up += (int64_t)(B.nr + B.nc) * r;
    }
    Blob b6;
    const size_t om = b6.add(md);
    cu.stage(b6);
    ge.stage(b6, &split);
    const char* base6 = dp.upload(b6, st);
    const MaxAbsDesc* dmd = reinterpret_cast<const MaxAbsDesc*>(base6 + om);
    launch_maxabs(dmd, nb, dmax.as<double>(), st);
    cu.launch(base6, st);
    ge.launch(base6, st);
    launch_maxabs(dmd, nb, dmax.as<double>() + nb, st);
    double* hm = dp.host<double>((size_t)3 * nb);
    HIPCHK(hipMemcpyAsync(hm, dmax.p, (size_t)2 * nb * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hm + 2 * nb, u11, (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < nb; ++i)
      block_errors.push_back(BlockErr{br[i].p, br[i].bi, hr[i], hm[i], hm[2 * nb + i], hm[nb + i]});
  }
  const bool uvbf = sizeof(T) == 4 && opts.uv_bf16 != 0;
  if (uvbf) {   // bases rounded to bfloat16 once; everything below uses the rounded values
    CopyBatch<T, T> rnd;
    for (int i = 0; i < nb; ++i) {
      const Block& B = s.fronts[br[i].p].blocks[br[i].bi];
      if (hr[i] == 0) continue;
      auto c1 = cd<T, T>(br[i].U, B.nr, br[i].U, B.nr, B.nr, hr[i]);
      auto c2 = cd<T, T>(br[i].V, B.nc, br[i].V, B.nc, B.nc, hr[i]);
      c1.bf16 = c2.bf16 = 1;
      rnd.v.push_back(c1);
      rnd.v.push_back(c2);
    }
    Blob rb;
    rnd.stage(rb);
    const char* rbase = dp.upload(rb, st);
    rnd.launch(rbase, st);
  }
  // ---- phase B
  std::map<std::pair<int, int>, int> bidx;   // (front, block) -> br index
  for (int i = 0; i < nb; ++i) bidx[{br[i].p, br[i].bi}] = i;
  Blob b2;
  CopyBatch<T, T> cp;        // scratch U/V -> persistent, G initialisation
  std::vector<PotrfDesc<T>> leaves;
  GemmBatch<T> lg1, lg2;
  int Lmax = 0;
  int64_t g_tot = 0, t1_tot = 0;
  for (int p : Hs) {
    const Front& f = s.fronts[p];
    FN& x = fn[p];
    const int nt = (int)f.pp_tree.size();
    x.nodeU.assign(nt, nullptr); x.nodeV.assign(nt, nullptr); x.nodeK.assign(nt, nullptr);
    x.leafInv.assign(nt, nullptr); x.nodeR.assign(nt, 0);
    x.r_top = f.nf() > 0 ? hr[bidx[{p, 0}]] : 0;
    int depth = 0;
    for (auto& t : f.pp_tree) depth = std::max(depth, t.level + 1);
    std::vector<int> rml(depth, 0);
    for (int i = 0; i < nt; ++i) {
      const TreeNode& t = f.pp_tree[i];
      if (t.left >= 0) {
        const int r = hr[bidx[{p, t.block}]];
        x.nodeR[i] = r;
        rml[t.level] = std::max(rml[t.level], r);
        Lmax = std::max(Lmax, t.level + 1);
      }
    }
    x.col.assign(depth + 1, 0);
    x.col[0] = x.r_top;
    for (int l = 0; l < depth; ++l) x.col[l + 1] = x.col[l] + rml[l];
    x.w = x.col[depth];
    g_tot += (int64_t)f.npiv * x.w;
    for (auto& t : f.pp_tree)
      if (t.left < 0) t1_tot += (int64_t)t.size * x.w;
  }
  T* gall = arena.alloc_n<T>(g_tot);
  if (g_tot > 0) launch_fill<T>(gall, g_tot, (T)0, st);
  for (int p : Hs) {
    const Front& f = s.fronts[p];
    FN& x = fn[p];
    x.G = gall;
    gall += (int64_t)f.npiv * x.w;
    if (x.r_top > 0) {
      const BR& t = br[bidx[{p, 0}]];
      x.W = base_alloc((int64_t)f.nf() * x.r_top, uvbf);
      auto cw = cd<T, T>(t.U, f.nf(), x.W, f.nf(), f.nf(), x.r_top);
      cw.bf16 = uvbf ? 2 : 0;
      cp.v.push_back(cw);
      cp.v.push_back(cd<T, T>(t.V, f.npiv, x.G, f.npiv, f.npiv, x.r_top));   // V_top -> X columns
    }
    for (int i = 0; i < (int)f.pp_tree.size(); ++i) {
      const TreeNode& t = f.pp_tree[i];
      if (t.left < 0) {
        x.leafInv[i] = arena.alloc_n<T>((int64_t)t.size * t.size);
        PotrfDesc<T> d{};
        if (sampled) { d.A = ppleaf.at(p)[i]; d.lda = t.size; }
        else { d.A = x.F + t.off + (int64_t)t.off * x.ld; d.lda = x.ld; }
        d.n = t.size;
        d.Inv = x.leafInv[i]; d.ldi = t.size;
        leaves.push_back(d);
        continue;
      }
      const int r = x.nodeR[i];
      const BR& bb = br[bidx[{p, t.block}]];
      const TreeNode& a = f.pp_tree[t.left];
      const TreeNode& be = f.pp_tree[t.right];
      x.nodeU[i] = base_alloc((int64_t)be.size * r, uvbf);
      x.nodeV[i] = base_alloc((int64_t)a.size * r, uvbf);
      x.nodeK[i] = arena.alloc_n<T>((int64_t)4 * r * r);
      auto cu = cd<T, T>(bb.U, be.size, x.nodeU[i], be.size, be.size, r);
      auto cv = cd<T, T>(bb.V, a.size, x.nodeV[i], a.size, a.size, r);
      cu.bf16 = cv.bf16 = uvbf ? 2 : 0;
      cp.v.push_back(cu);
      cp.v.push_back(cv);
      const int c = x.col[t.level];
      cp.v.push_back(cd<T, T>(bb.V, a.size, x.G + a.off + (int64_t)c * f.npiv, f.npiv, a.size, r));
      cp.v.push_back(cd<T, T>(bb.U, be.size, x.G + be.off + (int64_t)c * f.npiv, f.npiv, be.size, r));
    }
  }
  // leaf solves on G:  G_leaf <- L^{-T} L^{-1} G_leaf
  scrB.grow(std::max<int64_t>(t1_tot, 1) * sizeof(T), &ms, retired);
  {
    T* tp = scrB.as<T>();
    for (int p : Hs) {
      const Front& f = s.fronts[p];
      FN& x = fn[p];
      if (x.w == 0) continue;
      for (int i = 0; i < (int)f.pp_tree.size(); ++i) {
        const TreeNode& t = f.pp_tree[i];
        if (t.left >= 0) continue;
        lg1.v.push_back(gd<T>(x.leafInv[i], t.size, 0, x.G + t.off, f.npiv, 0, tp, t.size, t.size, x.w, t.size, 1.0,
                              0.0, GF_A_LOWER));
        lg2.v.push_back(gd<T>(x.leafInv[i], t.size, 1, tp, t.size, 0, x.G + t.off, f.npiv, t.size, x.w, t.size, 1.0,
                              0.0, GF_A_UPPER));
        tp += (int64_t)t.size * x.w;
      }
    }
  }
  const size_t oleaf = b2.add(leaves);
  cp.stage(b2);
  lg1.stage(b2, &split);
  lg2.stage(b2, &split);
  const char* base2 = dp.upload(b2, st);
  cp.launch(base2, st);
  timed_potrf<T>(reinterpret_cast<const PotrfDesc<T>*>(base2 + oleaf), leaves, s.leaf, d_status.as<int>(), st);
  lg1.launch(base2, st);
  lg2.launch(base2, st);

  // ---- SMW sweep, deepest HODLR level first
  for (int l = Lmax - 1; l >= 0; --l) {
    struct NodeRef { int p, i, r, c; };
    std::vector<NodeRef> nodes;
    size_t nP = 0, nK = 0, nPa = 0, nQ = 0;
    for (int p : Hs) {
      const Front& f = s.fronts[p];
      for (int i = 0; i < (int)f.pp_tree.size(); ++i) {
        const TreeNode& t = f.pp_tree[i];
        if (t.left < 0 || t.level != l || fn[p].nodeR[i] == 0) continue;
        const int r = fn[p].nodeR[i], c = fn[p].col[l];
        nodes.push_back({p, i, r, c});
        nP += al((size_t)2 * r * (c + r) * sizeof(T));
        nK += al((size_t)6 * r * r * sizeof(double));
        nPa += al((size_t)2 * r * std::max(c, 1) * sizeof(double));
        nQ += al((size_t)2 * r * std::max(c, 1) * sizeof(double)) + al((size_t)2 * r * std::max(c, 1) * sizeof(T));
      }
    }
    if (nodes.empty()) continue;
    scrB.grow(nP + nK + nPa + nQ, &ms, retired);
    char* cb = static_cast<char*>(scrB.p);
    auto tk = [&](size_t bytes) { char* r = cb; cb += al(bytes); return r; };
    Blob b3;
    GemmBatch<T> gP, gC;
    GemmBatch<double> gQ, gM, gX1, gX2;
    std::vector<CapDesc<T>> capd;
    std::vector<InvDesc> invd;
    CopyBatch<double, T> cQ, cK;
    for (auto& nr : nodes) {
      const Front& f = s.fronts[nr.p];
      FN& x = fn[nr.p];
      const TreeNode& t = f.pp_tree[nr.i];
      const TreeNode& a = f.pp_tree[t.left];
      const TreeNode& be = f.pp_tree[t.right];
      const int r = nr.r, c = nr.c, n2 = 2 * r;
      T* P = reinterpret_cast<T*>(tk((size_t)n2 * (c + r) * sizeof(T)));
      double* Kinv = reinterpret_cast<double*>(tk((size_t)6 * r * r * sizeof(double)));
      double* A64 = Kinv + (size_t)n2 * n2;
      double* B64 = A64 + (size_t)r * r;
      double* Pa = reinterpret_cast<double*>(tk((size_t)n2 * std::max(c, 1) * sizeof(double)));
      double* Q64 = reinterpret_cast<double*>(tk((size_t)n2 * std::max(c, 1) * sizeof(double)));
      T* Q = reinterpret_cast<T*>(tk((size_t)n2 * std::max(c, 1) * sizeof(T)));
      // P = [V^T G(alpha, 0:c+r); U^T G(beta, 0:c+r)]
      const BR& nb_ = br[bidx.at({nr.p, t.block})];     // the level's (rounded) bases
      gP.v.push_back(gd<T>(nb_.V, a.size, 1, x.G + a.off, f.npiv, 0, P, n2, r, c + r, a.size, 1.0, 0.0));
      gP.v.push_back(gd<T>(nb_.U, be.size, 1, x.G + be.off, f.npiv, 0, P + r, n2, r, c + r, be.size, 1.0,
                           0.0));
      CapDesc<T> cdsc{};
      cdsc.P = P; cdsc.ldp = n2; cdsc.r = r; cdsc.c = c; cdsc.Kinv = Kinv; cdsc.A = A64; cdsc.B = B64;
      cdsc.Pa = Pa;
      capd.push_back(cdsc);
      // K^{-1} = [[-B M, I + B M A], [M, -M A]], M = (I - A B)^{-1} built in Kinv(r:2r, 0:r)
      double* M = Kinv + r;
      gM.v.push_back(gd<double>(A64, r, 0, B64, r, 0, M, n2, r, r, r, -1.0, 1.0));
      InvDesc iv{};
      iv.A = M; iv.n = r; iv.ld = n2;
      invd.push_back(iv);
      gX1.v.push_back(gd<double>(B64, r, 0, M, n2, 0, Kinv, n2, r, r, r, -1.0, 0.0));                 // -B M
      gX1.v.push_back(gd<double>(M, n2, 0, A64, r, 0, Kinv + r + (size_t)r * n2, n2, r, r, r, -1.0, 0.0));  // -M A
      gX2.v.push_back(gd<double>(Kinv, n2, 0, A64, r, 0, Kinv + (size_t)r * n2, n2, r, r, r, -1.0, 1.0));  // I + B M A
      if (c > 0) {
        gQ.v.push_back(gd<double>(Kinv, n2, 0, Pa, n2, 0, Q64, n2, n2, c, n2, 1.0, 0.0));
        cQ.v.push_back(cd<double, T>(Q64, n2, Q, n2, n2, c));
        // G(alpha, 0:c) -= Y_alpha Q(0:r, :) ; G(beta, 0:c) -= Y_beta Q(r:2r, :)
        gC.v.push_back(gd<T>(x.G + a.off + (int64_t)c * f.npiv, f.npiv, 0, Q, n2, 0, x.G + a.off, f.npiv, a.size, c,
                             r, -1.0, 1.0));
        gC.v.push_back(gd<T>(x.G + be.off + (int64_t)c * f.npiv, f.npiv, 0, Q + r, n2, 0, x.G + be.off, f.npiv,
                             be.size, c, r, -1.0, 1.0));
      }
      cK.v.push_back(cd<double, T>(Kinv, n2, x.nodeK[nr.i], n2, n2, n2));
    }
    gP.stage(b3, &split);
    const size_t ocap = b3.add(capd), oinv = b3.add(invd);
    gM.stage(b3, &split);
    gX1.stage(b3, &split);
    gX2.stage(b3, &split);
    gQ.stage(b3, &split);
    cQ.stage(b3);
    gC.stage(b3, &split);
    cK.stage(b3);
    const char* base3 = dp.upload(b3, st);
    gP.launch(base3, st);
    launch_cap<T>(reinterpret_cast<const CapDesc<T>*>(base3 + ocap), (int)capd.size(), st);
    gM.launch(base3, st);
    {
      double fl = 0, by = 0;     // in-place Gauss-Jordan: n steps of an n x n rank-1 update
      int nmax = 0;
      for (const auto& d : invd) {
        fl += 2.0 * d.n * (double)d.n * d.n;
        by += 8.0 * 2.0 * d.n * (double)d.n;
        nmax = std::max(nmax, d.n);
      }
      const int id = prof_begin(gj_kind(nmax), st, fl, by);
      launch_gj_inverse(reinterpret_cast<const InvDesc*>(base3 + oinv), (int)invd.size(), nmax, d_status.as<int>(),
                        st);
      prof_end(id, st);
    }
    gX1.launch(base3, st);
    gX2.launch(base3, st);
    gQ.launch(base3, st);
    cQ.launch(base3, st);
    gC.launch(base3, st);
    cK.launch(base3, st);
  }

  // ---- Schur complement update of the ff part:  U_p = F_ff^HODLR - W S W^T
  {
    size_t need2 = 0;
    for (int p : Hs) {
      const Front& f = s.fronts[p];
      const int r = fn[p].r_top;
      if (r == 0) continue;
      need2 += al((size_t)f.npiv * r * 8) * 2 + al((size_t)f.nf() * r * 8) * 2 + al((size_t)r * r * 8) +
               al((size_t)f.nf() * r * sizeof(T));
    }
    scrB.grow(std::max<size_t>(need2, 256), &ms, retired);
    char* cb = static_cast<char*>(scrB.p);
    auto tk = [&](size_t bytes) { char* r = cb; cb += al(bytes); return r; };
    Blob b4;
    CopyBatch<T, double> c64;
    GemmBatch<double> gS, gWt;
    CopyBatch<double, T> cW;
    GemmBatch<T> gff, gup;
    for (int p : Hs) {
      const Front& f = s.fronts[p];
      FN& x = fn[p];
      const int npv = f.npiv, nf = f.nf();
      // F_ff off-diagonal blocks <- U V^T (compressed form, written densely for
      // the parent; a sampled front keeps U and V instead)
      for (int bi = 0; bi < (int)f.blocks.size() && !sampled; ++bi) {
        const Block& B = f.blocks[bi];
        if (B.kind != 2) continue;
        const BR& bb = br[bidx[{p, bi}]];
        gff.v.push_back(gd<T>(bb.U, B.nr, 0, bb.V, B.nc, 1, x.F + B.r0 + (int64_t)B.c0 * x.ld, x.ld, B.nr, B.nc,
                              hr[bidx[{p, bi}]], 1.0, 0.0));
      }
      const int r = x.r_top;
      if (r == 0) continue;
      const BR& tb = br[bidx[{p, 0}]];
      double* V64 = reinterpret_cast<double*>(tk((size_t)npv * r * 8));
      double* X64 = reinterpret_cast<double*>(tk((size_t)npv * r * 8));
      double* W64 = reinterpret_cast<double*>(tk((size_t)nf * r * 8));
      double* Wt64 = reinterpret_cast<double*>(tk((size_t)nf * r * 8));
      double* S64 = reinterpret_cast<double*>(tk((size_t)r * r * 8));
      T* Wt = reinterpret_cast<T*>(tk((size_t)nf * r * sizeof(T)));
      if (sampled) x.Wt = Wt = keep_alloc(p, (int64_t)nf * r);
      c64.v.push_back(cd<T, double>(tb.V, npv, V64, npv, npv, r));
      c64.v.push_back(cd<T, double>(x.G, npv, X64, npv, npv, r));
      c64.v.push_back(cd<T, double>(tb.U, nf, W64, nf, nf, r));
      gS.v.push_back(gd<double>(V64, npv, 1, X64, npv, 0, S64, r, r, r, npv, 1.0, 0.0));       // S = V^T X
      gWt.v.push_back(gd<double>(W64, nf, 0, S64, r, 0, Wt64, nf, nf, r, r, 1.0, 0.0));        // W S
      cW.v.push_back(cd<double, T>(Wt64, nf, Wt, nf, nf, r));
      if (!sampled)
        gup.v.push_back(gd<T>(Wt, nf, 0, tb.U, nf, 1, x.F + npv + (int64_t)npv * x.ld, x.ld, nf, nf, r, -1.0, 1.0,
                            GF_LOWER_C));
    }
    c64.stage(b4);
    gS.stage(b4, &split);
    gWt.stage(b4, &split);
    cW.stage(b4);
    gff.stage(b4, &split);
    gup.stage(b4, &split);
    const char* base4 = dp.upload(b4, st);
    c64.launch(base4, st);
    gS.launch(base4, st);
    gWt.launch(base4, st);
    cW.launch(base4, st);
    gff.launch(base4, st);
    gup.launch(base4, st);
  }
  if (!sampled) return;
  // ---- what the parents read of a sampled front: F_ff^HODLR as its cluster
  // tree (leaf blocks gathered above, each internal node's U and V), root first
  Blob b5;
  CopyBatch<T, T> kc;
  std::vector<FfNode> nodes;
  std::vector<std::pair<int, size_t>> first;
  for (int p : Hs) {
    const Front& f = s.fronts[p];
    if (f.ff_tree.empty()) continue;
    int64_t tot = 0;
    for (const TreeNode& t : f.ff_tree)
      if (t.left >= 0) tot += (int64_t)t.size * hr[bidx.at({p, t.block})];
    T* kp = tot > 0 ? keep_alloc(p, tot) : nullptr;
    first.push_back({p, nodes.size()});
    for (size_t k = 0; k < f.ff_tree.size(); ++k) {
      const TreeNode& t = f.ff_tree[k];
      FfNode nd{};
      nd.off = t.off - f.npiv; nd.size = t.size; nd.left = t.left; nd.right = t.right;
      if (t.left < 0) {
        nd.U = ffleaf.at(p)[k];
      } else {
        const BR& bb = br[bidx.at({p, t.block})];
        const int r = hr[bidx.at({p, t.block})];
        const TreeNode& a = f.ff_tree[t.left];
        const TreeNode& be = f.ff_tree[t.right];
        nd.rank = r;
        if (r > 0) {   // U: rows in the right child; V: rows in the left child
          T* U = kp;
          T* V = kp + (int64_t)be.size * r;
          kp += (int64_t)t.size * r;
          kc.v.push_back(cd<T, T>(bb.U, be.size, U, be.size, be.size, r));
          kc.v.push_back(cd<T, T>(bb.V, a.size, V, a.size, a.size, r));
          nd.U = U;
          nd.V = V;
        }
      }
      nodes.push_back(nd);
    }
  }
  const size_t on = b5.add(nodes);
  kc.stage(b5);
  const char* base5 = dp.upload(b5, st);
  kc.launch(base5, st);
  for (auto& w : first) fn[w.first].ffnodes = reinterpret_cast<const FfNode*>(base5 + on) + w.second;
}

// ================================================================ apply ====
template <typename T>
typename Numeric<T>::Layout Numeric<T>::plan_layout(int nrhs) const {
  const Symbolic& s = *sym;
  const int nfr = (int)s.fronts.size();
  Layout L;
  L.t_off.resize(nfr); L.z_off.resize(nfr); L.h_off.resize(nfr);
  L.q_off.resize(nfr); L.l_off.resize(nfr);
  // workspace layout (elements of T); x in the permuted order comes first
  int64_t tot = (int64_t)s.n * nrhs;
  for (int p = 0; p < nfr; ++p) {
    const Front& f = s.fronts[p];
    L.t_off[p] = tot; tot += (int64_t)f.n() * nrhs;
    // a HODLR front's z is its t's pivot rows (read by X^T t before the
    // leaf solves change them in place); a dense front's z is separate
    if (fn[p].dense) { L.z_off[p] = tot; tot += (int64_t)f.npiv * nrhs; }
    else L.z_off[p] = L.t_off[p];
    if (!fn[p].dense) {
      L.h_off[p] = tot; tot += (int64_t)std::max(fn[p].r_top, 1) * nrhs;
      L.q_off[p].assign(f.pp_tree.size(), 0);
      L.l_off[p].assign(f.pp_tree.size(), 0);
      for (size_t i = 0; i < f.pp_tree.size(); ++i) {
        const TreeNode& t = f.pp_tree[i];
        if (t.left >= 0) { L.q_off[p][i] = tot; tot += (int64_t)4 * std::max(fn[p].nodeR[i], 1) * nrhs; }
        else { L.l_off[p][i] = tot; tot += (int64_t)t.size * nrhs; }
      }
    }
  }
  L.tot = tot;
  return L;
}

template <typename T>
typename Numeric<T>::Plan* Numeric<T>::get_plan(int nrhs) {
  auto it = plans.find(nrhs);
  if (it != plans.end()) return it->second.get();
  auto pl = std::make_unique<Plan>();
  pl->dp.ar.ms = &ms;
  const Layout L = plan_layout(nrhs);
  pl->work.alloc(L.tot * sizeof(T), &ms);
  pl->split.alloc(kSplitPlanBytes, &ms);
  Plan* raw = pl.get();
  build_plan(*raw, nrhs, L, raw->work.template as<T>(), raw->split.template as<T>(), kSplitPlanBytes / sizeof(T),
             [this, raw](Blob& bl) { return raw->dp.upload(bl, st); });
  HIPCHK(hipStreamSynchronize(st));
  plans[nrhs] = std::move(pl);
  return raw;
}

// The apply's step sequence for nrhs right-hand sides: workspace wk
// (L.tot elements), split-K partial sums in part (cap elements), and the
// descriptor blobs placed on the device by `upload`.
template <typename T>
template <typename Upload>
void Numeric<T>::build_plan(Plan& plan, int nrhs, const Layout& L, T* wk, T* part, size_t cap, Upload&& upload) {
  const Symbolic& s = *sym;
  Plan* pl = &plan;
  pl->nrhs = nrhs;
  const int bff = (sizeof(T) == 4 && opts.uv_bf16) ? GF_A_BF16 : 0;   // U, V, W kept in bfloat16
  const int nfr = (int)s.fronts.size();
  const int N = s.n;
  const std::vector<int64_t>&t_off = L.t_off, &z_off = L.z_off, &h_off = L.h_off;
  const std::vector<std::vector<int64_t>>&q_off = L.q_off, &l_off = L.l_off;
  pl->xn = wk;
  Blob b;
  const int chunk_min = opts.apply_split_chunk > 0 ? opts.apply_split_chunk : kSplitChunk;
  std::unordered_set<const T*> foldable;   // B arrays read by one product only, right after their writers
  // the partial-sum area of a batch starts at `off` (past partials that it reads)
  auto stage_gemm = [&](GemmBatch<T>& g, size_t off) {
    g.stage(b, off < cap ? part + off : nullptr, off < cap ? cap - off : 0, chunk_min, opts.apply_split_target);
  };
  auto push_gemm = [&](GemmBatch<T>& g) {
    if (g.n && g.nfold) pl->recs.push_back({5, g.off, g.n, g.tiles, g.flops, g.bytes, g.tn, g.foff});
    else if (g.n) pl->recs.push_back({0, g.off, g.n, g.tiles, g.flops, g.bytes, g.tn});
    if (g.rn) pl->recs.push_back({4, g.roff, g.rn, g.rtiles, 0.0, g.rbytes});
  };
  auto rec_gemm = [&](GemmBatch<T>& g) {
    stage_gemm(g, 0);
    push_gemm(g);
  };
  // c runs right after p and its descriptors marked by fold_b read outputs of p
  // that nothing reads later: those outputs' split-K partials are summed
  // while c loads its B operand, and their reduction launch is left out
  auto rec_pair = [&](GemmBatch<T>& p, GemmBatch<T>& c) {
    stage_gemm(p, 0);
    stage_gemm(c, p.pused);
    std::vector<const T*> folded;
    c.resolve_folds(p, foldable, b, folded);
    p.drop_reductions(b, folded);
    push_gemm(p);
    push_gemm(c);
  };
  // marks a product whose B (u2: h_p, g2: q, d2: h_p or z) is written by
  // the batch just before it and read by nothing after it
  auto fold_b = [&](GemmDesc<T> g) {
    foldable.insert(g.B);
    return g;
  };
  auto rec_copy = [&](CopyBatch<T, T>& c) {
    c.stage(b);
    if (c.n) pl->recs.push_back({1, c.off, c.n, c.tiles});
  };
  const int H = (int)s.levels.size();
  // upward pass
  for (int h = 0; h < H; ++h) {
    std::vector<VecAsmDesc<T>> va;
    GemmBatch<T> u1, u2, lf1, lf2;
    int Lmax = 0;
    for (int p : s.levels[h]) {
      const Front& f = s.fronts[p];
      const FN& x = fn[p];
      VecAsmDesc<T> d{};
      d.t = wk + t_off[p]; d.xs = pl->xn + f.start; d.nhat = f.n(); d.npiv = f.npiv; d.ldt = f.n(); d.ldx = N;
      d.nchild = (int)f.children.size();
      for (int ci = 0; ci < d.nchild && ci < 2; ++ci) {
        const int c = f.children[ci];
        const Front& fc = s.fronts[c];
        d.ct[ci] = wk + t_off[c]; d.crel[ci] = fc.relmap.empty() ? nullptr : d_relmap.as<int>() + relmap_off[c];
        d.cnp[ci] = fc.npiv; d.cnf[ci] = fc.nf(); d.cld[ci] = fc.n();
      }
      va.push_back(d);
      T* t = wk + t_off[p];
      T* z = wk + z_off[p];
      const int np = f.npiv, nf = f.nf(), nh = f.n();
      if (x.dense) {
        u1.v.push_back(gd<T>(x.Linv, np, 0, t, nh, 0, z, np, np, nrhs, np, 1.0, 0.0, GF_A_LOWER));
        if (nf > 0) u2.v.push_back(gd<T>(x.Lfp, nf, 0, z, np, 0, t + np, nh, nf, nrhs, np, -1.0, 1.0));
      } else {
        T* hb = wk + h_off[p];
        if (x.r_top > 0) {
          u1.v.push_back(gd<T>(x.G, np, 1, t, nh, 0, hb, x.r_top, x.r_top, nrhs, np, 1.0, 0.0));   // X^T t_p
          u2.v.push_back(fold_b(gd<T>(x.W, nf, 0, hb, x.r_top, 0, t + np, nh, nf, nrhs, x.r_top, -1.0, 1.0, bff)));
        }
        for (size_t i = 0; i < f.pp_tree.size(); ++i) {
          const TreeNode& tn = f.pp_tree[i];
          if (tn.left >= 0) { Lmax = std::max(Lmax, tn.level + 1); continue; }
          T* T1 = wk + l_off[p][i];
          lf1.v.push_back(gd<T>(x.leafInv[i], tn.size, 0, z + tn.off, nh, 0, T1, tn.size, tn.size, nrhs, tn.size, 1.0,
                                0.0, GF_A_LOWER));
          lf2.v.push_back(gd<T>(x.leafInv[i], tn.size, 1, T1, tn.size, 0, z + tn.off, nh, tn.size, nrhs, tn.size, 1.0,
                                0.0, GF_A_UPPER));
        }
      }
    }
    {
      size_t o = b.add(va);
      pl->recs.push_back({2, o, (int)va.size(), 0});
    }
    // u2 (rows np.. of t, after u1) and lf1 (reads the pivot rows of t,
    // after u1 has read them) touch different memory, so they share a launch
    lf1.v.insert(lf1.v.end(), u2.v.begin(), u2.v.end());
    rec_pair(u1, lf1);
    rec_gemm(lf2);
    for (int l = Lmax - 1; l >= 0; --l) {
      GemmBatch<T> g1, g2, g3;
      for (int p : s.levels[h]) {
        if (fn[p].dense) continue;
        const Front& f = s.fronts[p];
        const FN& x = fn[p];
        T* z = wk + z_off[p];
        const int np = f.npiv, zl = f.n();
        for (size_t i = 0; i < f.pp_tree.size(); ++i) {
          const TreeNode& t = f.pp_tree[i];
          if (t.left < 0 || t.level != l || x.nodeR[i] == 0) continue;
          const TreeNode& a = f.pp_tree[t.left];
          const TreeNode& be = f.pp_tree[t.right];
          const int r = x.nodeR[i], n2 = 2 * r, c = x.col[l];
          T* q = wk + q_off[p][i];
          T* q2 = q + (int64_t)n2 * nrhs;
          g1.v.push_back(gd<T>(x.nodeV[i], a.size, 1, z + a.off, zl, 0, q, n2, r, nrhs, a.size, 1.0, 0.0, bff));
          g1.v.push_back(gd<T>(x.nodeU[i], be.size, 1, z + be.off, zl, 0, q + r, n2, r, nrhs, be.size, 1.0, 0.0, bff));
          g2.v.push_back(fold_b(gd<T>(x.nodeK[i], n2, 0, q, n2, 0, q2, n2, n2, nrhs, n2, 1.0, 0.0)));
          g3.v.push_back(gd<T>(x.G + a.off + (int64_t)c * np, np, 0, q2, n2, 0, z + a.off, zl, a.size, nrhs, r, -1.0,
                               1.0));
          g3.v.push_back(gd<T>(x.G + be.off + (int64_t)c * np, np, 0, q2 + r, n2, 0, z + be.off, zl, be.size, nrhs, r,
                               -1.0, 1.0));
        }
      }
      rec_pair(g1, g2);
      rec_gemm(g3);
    }
  }
  // downward pass.  Every HODLR front's z is final after the upward pass:
  // one launch copies them all into x, where the downward corrections then
  // accumulate directly
  {
    CopyBatch<T, T> zx;
    for (int p = 0; p < nfr; ++p) {
      const Front& f = s.fronts[p];
      if (fn[p].dense || f.npiv == 0) continue;
      zx.v.push_back(cd<T, T>(wk + z_off[p], f.n(), pl->xn + f.start, N, f.npiv, nrhs));
    }
    rec_copy(zx);
  }
  for (int h = H - 1; h >= 0; --h) {
    // t_f = x(I_p^f) is read by the first product through the front's
    // update set (a row map on its B operand), so it is never formed
    std::map<int, const int*> upd_dev;
    {
      std::vector<int> upd;
      std::vector<std::pair<int, int64_t>> uo;
      for (int p : s.levels[h]) {
        const Front& f = s.fronts[p];
        if (f.nf() == 0) continue;
        uo.push_back({p, (int64_t)upd.size()});
        upd.insert(upd.end(), f.upd.begin(), f.upd.end());
      }
      if (!upd.empty()) {
        Blob ub;
        const size_t o = ub.add(upd);
        const char* ubase = upload(ub);
        for (auto& q : uo) upd_dev[q.first] = reinterpret_cast<const int*>(ubase + o) + q.second;
      }
    }
    GemmBatch<T> d1, d2;
    for (int p : s.levels[h]) {
      const Front& f = s.fronts[p];
      const FN& x = fn[p];
      const int np = f.npiv, nf = f.nf();
      T* z = wk + z_off[p];
      if (x.dense) {
        if (nf > 0) {
          auto g = gd<T>(x.Lfp, nf, 1, pl->xn, N, 0, z, np, np, nrhs, nf, -1.0, 1.0);
          g.brow = upd_dev.at(p);
          d1.v.push_back(g);
        }
        d2.v.push_back(fold_b(gd<T>(x.Linv, np, 1, z, np, 0, pl->xn + f.start, N, np, nrhs, np, 1.0, 0.0, GF_A_UPPER)));
      } else {
        T* hb = wk + h_off[p];
        if (x.r_top > 0) {
          auto g = gd<T>(x.W, nf, 1, pl->xn, N, 0, hb, x.r_top, x.r_top, nrhs, nf, 1.0, 0.0, bff);
          g.brow = upd_dev.at(p);
          d1.v.push_back(g);
          d2.v.push_back(fold_b(gd<T>(x.G, np, 0, hb, x.r_top, 0, pl->xn + f.start, N, np, nrhs, x.r_top, -1.0, 1.0)));
        }
      }
    }
    rec_pair(d1, d2);
  }
  pl->desc = upload(b);
}

template <typename T>
void Numeric<T>::apply(int nrhs, const double* r, double* z, hipStream_t stream) {
  hipStream_t keep = st;
  st = stream;
  Plan* pl = get_plan(nrhs);
  st = keep;
  const int N = sym->n;
  launch_perm_in<T>(r, pl->xn, d_perm.as<int>(), N, nrhs, stream);
  // the apply_graph-th apply with this count records the graph (recording
  // costs about as much as a few direct applies).  Its nodes are recorded
  // untimed: while a timing session runs, only the direct applies (and the
  // factorization's launches) are timed, and the replays run as they would
  // without it.
  ++pl->uses;
  bool replay = opts.apply_graph > 0 && pl->uses >= opts.apply_graph && !pl->no_graph;
  if (replay && !pl->exec) {
    // record the step sequence once on a stream of this handle; the plan's
    // buffers and descriptors stay put, so the graph stays valid with it
    hipGraph_t g = nullptr;
    bool ok = cap || hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      prof_suspend(true);
      try {
        launch_recs(*pl, cap);
      } catch (...) {   // never leave the stream capturing
        prof_suspend(false);
        if (hipStreamEndCapture(cap, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        pl->no_graph = true;
        throw;
      }
      prof_suspend(false);
      ok = hipStreamEndCapture(cap, &g) == hipSuccess && g;
      ok = ok && hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0) == hipSuccess;
      if (g) (void)hipGraphDestroy(g);
    }
    if (!ok) {
      (void)hipGetLastError();
      pl->exec = nullptr;
      pl->no_graph = true;
      replay = false;
    }
  }
  if (replay) HIPCHK(hipGraphLaunch(pl->exec, stream));
  else launch_recs(*pl, stream);
  launch_perm_out<T>(pl->xn, z, d_iperm.as<int>(), N, nrhs, stream);
  HIPCHK(hipGetLastError());
}

// The same step sequence as apply(), with its memory in the device's
// scratch: workspace first, split-K partials next, descriptors after them.
// The descriptors are uploaded again (host planning and a blocking copy)
// whenever the scratch last held another handle's plan or another nrhs.
template <typename T>
void Numeric<T>::apply_noalloc(int nrhs, const double* r, double* z, hipStream_t stream) {
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != device) throw Err{MF_ESTATE, "the factor's device is not the current device"};
  ScratchState& S = scratch_state(device);
  std::lock_guard<std::mutex> g(S.mu);
  char* base = scratch_address(S);
  const Layout L = plan_layout(nrhs);
  const size_t wbytes = ((size_t)L.tot * sizeof(T) + 255) & ~size_t(255);
  if (wbytes + kSplitPlanBytes >= (size_t)MF_APPLY_SCRATCH_BYTES)
    throw Err{MF_EINVAL, "the apply workspace for " + std::to_string(nrhs) + " right-hand sides needs " +
                             std::to_string(wbytes) + " bytes; the scratch holds " +
                             std::to_string((size_t)MF_APPLY_SCRATCH_BYTES - kSplitPlanBytes)};
  if (!na_plan || S.owner != uid || S.nrhs != nrhs) {
    S.owner = 0;
    na_plan.reset();
    auto pl = std::make_unique<Plan>();
    char* bump = base + wbytes + kSplitPlanBytes;
    char* const end = base + MF_APPLY_SCRATCH_BYTES;
    auto up = [&](Blob& bl) -> char* {
      const size_t n = bl.h.size();
      if (n == 0) return nullptr;
      if (n > (size_t)(end - bump))
        throw Err{MF_EINVAL, "the apply descriptors do not fit the scratch next to the workspace"};
      char* d = bump;
      bump += (n + 255) & ~size_t(255);
      HIPCHK(hipMemcpyAsync(d, bl.h.data(), n, hipMemcpyHostToDevice, stream));
      HIPCHK(hipStreamSynchronize(stream));   // the host blob may go now
      return d;
    };
    build_plan(*pl, nrhs, L, reinterpret_cast<T*>(base), reinterpret_cast<T*>(base + wbytes),
               kSplitPlanBytes / sizeof(T), up);
    na_plan = std::move(pl);
    S.owner = uid;
    S.nrhs = nrhs;
  }
  const int N = sym->n;
  launch_perm_in<T>(r, na_plan->xn, d_perm.as<int>(), N, nrhs, stream);
  launch_recs(*na_plan, stream);
  launch_perm_out<T>(na_plan->xn, z, d_iperm.as<int>(), N, nrhs, stream);
  HIPCHK(hipGetLastError());
}

template <typename T>
void Numeric<T>::launch_recs(const Plan& plan, hipStream_t stream) {
  const Plan* pl = &plan;
  const int N = sym->n, nrhs = pl->nrhs;
  for (const Rec& rc : pl->recs) {
    const char* base = pl->desc + rc.off;
    switch (rc.kind) {
      case 0: {
        const int id = prof_begin(pk<T>(rc.tn == kTileNarrow ? PK_GEMMN_F64 : PK_GEMM_F64), stream, rc.flops,
                                  rc.bytes);
        launch_gemm<T>(reinterpret_cast<const GemmDesc<T>*>(base), rc.n, rc.tiles, stream, rc.tn);
        prof_end(id, stream);
        break;
      }
      case 5: {
        const int id = prof_begin(pk<T>(PK_GEMMNF_F64), stream, rc.flops, rc.bytes);
        launch_gemm_fold<T>(reinterpret_cast<const GemmDesc<T>*>(base),
                            reinterpret_cast<const FoldDesc<T>*>(pl->desc + rc.off2), rc.n, rc.tiles, stream);
        prof_end(id, stream);
        break;
      }
      case 4: {
        const int id = prof_begin(pk<T>(PK_GEMM_REDUCE_F64), stream, 0.0, rc.bytes);
        launch_gemm_reduce<T>(reinterpret_cast<const GemmDesc<T>*>(base), rc.n, rc.tiles, stream);
        prof_end(id, stream);
        break;
      }
      case 1: launch_copy<T, T>(reinterpret_cast<const CopyDesc<T, T>*>(base), rc.n, rc.tiles, stream); break;
      case 2: launch_vec_asm<T>(reinterpret_cast<const VecAsmDesc<T>*>(base), rc.n, nrhs, stream); break;
    }
  }
}

void NumericBase::note_stream(hipStream_t st) {
  std::lock_guard<std::mutex> g(ev_mu);
  // a failed record is dropped here, not left for the next hipGetLastError
  for (auto& e : stream_events)
    if (e.first == st) {
      if (hipEventRecord(e.second, st) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(st);
        (void)hipGetLastError();
      }
      return;
    }
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(st);
    (void)hipGetLastError();
    return;
  }
  if (hipEventRecord(ev, st) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(st);
    (void)hipGetLastError();
  }
  stream_events.push_back({st, ev});
}

void NumericBase::wait_streams() {
  std::lock_guard<std::mutex> g(ev_mu);
  for (auto& e : stream_events) {
    if (hipEventSynchronize(e.second) != hipSuccess) (void)hipGetLastError();
    (void)hipEventDestroy(e.second);
  }
  stream_events.clear();
}

// ================================================================ GMRES ====
void NumericBase::spmv(int nrhs, const double* x, double* y, double alpha, double beta, hipStream_t st,
                       const int* win) {
  // CSR read once, x gathered once per right-hand side, y written (and read)
  const double by = 12.0 * sym->nnz + 4.0 * (sym->n + 1) + 8.0 * sym->n * nrhs * (beta != 0.0 ? 3.0 : 2.0);
  const int id = prof_begin(PK_SPMV, st, 2.0 * sym->nnz * nrhs, by);
  launch_spmv(d_rowptr.as<int>(), d_colind.as<int>(), d_vals.as<double>(), x, y, sym->n, nrhs, alpha, beta, st,
              win);
  prof_end(id, st);
}

void NumericBase::gmres(int nrhs, const double* b, double* x, double tol, const mf_gmres_opts& o,
                        mf_gmres_info* info_out, mf_status* st_out, const int32_t* win_host) {
  hipStream_t st = static_cast<hipStream_t>(o.stream);
  const int N = sym->n, m = std::max(1, o.restart);
  const int64_t vs = (int64_t)N * nrhs;
  g_V.ensure((size_t)(m + 1) * vs * 8, &ms, st);
  g_Z.ensure((size_t)m * vs * 8, &ms, st);
  g_w.ensure((size_t)vs * 8, &ms, st);
  g_r.ensure((size_t)vs * 8, &ms, st);
  const int nsmall = 3 * (m + 2) * nrhs + 4 * nrhs;
  g_small.ensure((size_t)nsmall * 8 + (win_host ? (size_t)2 * nrhs * 4 : 0), &ms, st);
  int* win = nullptr;             // column row windows on the device, after the doubles
  if (win_host) {
    win = reinterpret_cast<int*>(g_small.as<double>() + nsmall);
    PinnedScratch wp((size_t)2 * nrhs * 4, st);
    std::copy(win_host, win_host + 2 * nrhs, wp.as<int>(0));
    HIPCHK(hipMemcpyAsync(win, wp.as<int>(0), (size_t)2 * nrhs * 4, hipMemcpyHostToDevice, st));
  }
  g_partial.ensure((size_t)mdot_chunks(nrhs) * (m + 2) * nrhs * 8, &ms, st);
  double* V = g_V.as<double>();
  double* Z = g_Z.as<double>();
  double* w = g_w.as<double>();
  double* r = g_r.as<double>();
  double* sm = g_small.as<double>();
  double* h1 = sm;                        // (m+1) x nrhs
  double* h2 = sm + (m + 1) * nrhs;       // (m+1) x nrhs
  double* nr2 = sm + 2 * (m + 1) * nrhs;  // nrhs
  double* ydev = nr2 + nrhs;              // m x nrhs
  double* part = g_partial.as<double>();

  // host sides of the small transfers in pinned memory, so they are queued
  // copies; every one is followed by a synchronisation before the host
  // touches the buffer again
  const size_t nhs = (size_t)2 * (m + 1) * nrhs + nrhs, nys = (size_t)m * nrhs;
  PinnedScratch pin((nhs + nrhs + nys) * sizeof(double), st);
  double* hs = pin.as<double>(0);
  double* nrm2_h = hs + nhs;
  double* ybuf_h = nrm2_h + nrhs;
  auto read_small = [&](int count) {
    HIPCHK(hipMemcpyAsync(hs, sm, count * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  };
  // ||b||
  launch_mdot(b, 0, 1, b, N, nrhs, part, nr2, 0, st, win);
  HIPCHK(hipMemcpyAsync(hs, nr2, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<double> bnorm(nrhs), beta(nrhs);
  for (int k = 0; k < nrhs; ++k) bnorm[k] = std::sqrt(hs[k]);
  launch_fill<double>(x, vs, 0.0, st);
  launch_axpby(b, b, r, 1.0, 0.0, vs, st);
  beta = bnorm;
  std::vector<int> iters(nrhs, 0), conv(nrhs, 0);
  std::vector<double> H((size_t)nrhs * (m + 1) * m), cs((size_t)nrhs * m), sn((size_t)nrhs * m),
      g((size_t)nrhs * (m + 1)), ybuf((size_t)m * nrhs);
  const int maxit = o.maxit;
  for (;;) {
    bool any = false;
    std::vector<double> nrm2(nrhs);
    for (int k = 0; k < nrhs; ++k) {
      if (beta[k] <= tol * bnorm[k]) conv[k] = 1;
      const bool act = !conv[k] && iters[k] < maxit;
      any |= act;
      nrm2[k] = act ? beta[k] * beta[k] : 0.0;   // inactive columns get a zero basis
    }
    if (!any) break;
    std::vector<char> act(nrhs);
    for (int k = 0; k < nrhs; ++k) act[k] = !conv[k] && iters[k] < maxit;
    std::copy(nrm2.begin(), nrm2.end(), nrm2_h);
    HIPCHK(hipMemcpyAsync(nr2, nrm2_h, nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    launch_scale_cols(r, V, nr2, N, nrhs, st, win);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    for (int k = 0; k < nrhs; ++k) g[(size_t)k * (m + 1)] = act[k] ? beta[k] : 0.0;
    int jend = 0;
    std::vector<int> jk(nrhs, 0);          // Arnoldi columns used by each rhs this cycle
    std::vector<char> frozen(nrhs, 0);
    for (int j = 0; j < m; ++j) {
      double* Vj = V + (int64_t)j * vs;
      double* Zj = Z + (int64_t)j * vs;
      apply(nrhs, Vj, Zj, st);
      spmv(nrhs, Zj, w, 1.0, 0.0, st, win);
      // classical Gram-Schmidt, twice
      launch_mdot(V, vs, j + 1, w, N, nrhs, part, h1, 0, st, win);
      launch_maxpy(V, vs, j + 1, h1, w, N, nrhs, -1.0, st, win);
      launch_mdot(V, vs, j + 1, w, N, nrhs, part, h2, 0, st, win);
      launch_maxpy(V, vs, j + 1, h2, w, N, nrhs, -1.0, st, win);
      launch_mdot(w, 0, 1, w, N, nrhs, part, nr2, 0, st, win);
      launch_scale_cols(w, V + (int64_t)(j + 1) * vs, nr2, N, nrhs, st, win);
      read_small(2 * (m + 1) * nrhs + nrhs);
      bool all_done = true;
      for (int k = 0; k < nrhs; ++k) {
        if (!act[k] || frozen[k]) continue;
        double* Hk = H.data() + (size_t)k * (m + 1) * m;   // column-major (m+1) x m
        double* gk = g.data() + (size_t)k * (m + 1);
        double* ck = cs.data() + (size_t)k * m;
        double* sk = sn.data() + (size_t)k * m;
        for (int i = 0; i <= j; ++i) Hk[i + (size_t)j * (m + 1)] = hs[i * nrhs + k] + hs[(m + 1) * nrhs + i * nrhs + k];
        Hk[(j + 1) + (size_t)j * (m + 1)] = std::sqrt(hs[2 * (m + 1) * nrhs + k]);
        for (int i = 0; i < j; ++i) {
          const double a = Hk[i + (size_t)j * (m + 1)], bb = Hk[i + 1 + (size_t)j * (m + 1)];
          Hk[i + (size_t)j * (m + 1)] = ck[i] * a + sk[i] * bb;
          Hk[i + 1 + (size_t)j * (m + 1)] = -sk[i] * a + ck[i] * bb;
        }
        const double a = Hk[j + (size_t)j * (m + 1)], bb = Hk[j + 1 + (size_t)j * (m + 1)];
        const double den = std::hypot(a, bb);
        ck[j] = den > 0 ? a / den : 1.0;
        sk[j] = den > 0 ? bb / den : 0.0;
        Hk[j + (size_t)j * (m + 1)] = den;
        Hk[j + 1 + (size_t)j * (m + 1)] = 0.0;
        gk[j + 1] = -sk[j] * gk[j];
        gk[j] = ck[j] * gk[j];
        iters[k]++;
        jk[k] = j + 1;
        const bool done = std::fabs(gk[j + 1]) <= tol * bnorm[k] || iters[k] >= maxit || den == 0.0;
        if (done) frozen[k] = 1;
        all_done &= done;
      }
      jend = j + 1;
      if (all_done) break;
    }
    // y = H^{-1} g per column; x += Z y
    std::fill(ybuf.begin(), ybuf.end(), 0.0);
    for (int k = 0; k < nrhs; ++k) {
      if (!act[k]) continue;
      const double* Hk = H.data() + (size_t)k * (m + 1) * m;
      const double* gk = g.data() + (size_t)k * (m + 1);
      const int kk = jk[k];
      for (int i = kk - 1; i >= 0; --i) {
        double sacc = gk[i];
        for (int c = i + 1; c < kk; ++c) sacc -= Hk[i + (size_t)c * (m + 1)] * ybuf[c * nrhs + k];
        const double d = Hk[i + (size_t)i * (m + 1)];
        ybuf[i * nrhs + k] = d != 0.0 ? sacc / d : 0.0;
      }
    }
    std::copy(ybuf.begin(), ybuf.begin() + (std::ptrdiff_t)jend * nrhs, ybuf_h);
    HIPCHK(hipMemcpyAsync(ydev, ybuf_h, (size_t)jend * nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    launch_xupdate(Z, vs, jend, ydev, x, N, nrhs, st, win);
    spmv(nrhs, x, w, 1.0, 0.0, st, win);
    launch_axpby(b, w, r, 1.0, -1.0, vs, st);
    launch_mdot(r, 0, 1, r, N, nrhs, part, nr2, 0, st, win);
    HIPCHK(hipMemcpyAsync(hs, nr2, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int k = 0; k < nrhs; ++k) beta[k] = std::sqrt(hs[k]);
  }
  bool ok = true;
  for (int k = 0; k < nrhs; ++k) {
    const bool c = conv[k] || beta[k] <= tol * bnorm[k];
    ok &= c;
    if (info_out) info_out[k] = {iters[k], c ? 1 : 0, bnorm[k] > 0 ? beta[k] / bnorm[k] : 0.0};
  }
  *st_out = ok ? MF_OK : MF_ENOCONV;
}

// ======================================================= direct solve ====
// The factor as a direct solver (Conclusion: at high accuracy, a standalone
// direct solver): x = M^{-1} b, then `refine` steps of iterative refinement
// x += M^{-1} (b - A x) with float64 residuals; the final true relative
// residuals go to info.
void NumericBase::direct_solve(int nrhs, const double* b, double* x, int refine, hipStream_t st,
                               mf_gmres_info* info_out) {
  const int N = sym->n;
  const int64_t vs = (int64_t)N * nrhs;
  g_r.ensure((size_t)vs * 8, &ms, st);
  g_w.ensure((size_t)vs * 8, &ms, st);
  g_small.ensure((size_t)2 * nrhs * 8, &ms, st);
  g_partial.ensure((size_t)mdot_chunks(nrhs) * nrhs * 8, &ms, st);
  double* r = g_r.as<double>();
  double* w = g_w.as<double>();
  double* nb = g_small.as<double>();
  double* nr = nb + nrhs;
  double* part = g_partial.as<double>();
  apply(nrhs, b, x, st);
  for (int s = 0; s < refine; ++s) {
    spmv(nrhs, x, w, 1.0, 0.0, st);
    launch_axpby(b, w, r, 1.0, -1.0, vs, st);       // r = b - A x
    apply(nrhs, r, w, st);
    launch_axpby(x, w, x, 1.0, 1.0, vs, st);        // x += M^{-1} r
  }
  spmv(nrhs, x, w, 1.0, 0.0, st);
  launch_axpby(b, w, r, 1.0, -1.0, vs, st);
  launch_mdot(r, 0, 1, r, N, nrhs, part, nr, 0, st);
  launch_mdot(b, 0, 1, b, N, nrhs, part, nb, 0, st);
  PinnedScratch pin((size_t)2 * nrhs * sizeof(double), st);
  double* h = pin.as<double>(0);
  HIPCHK(hipMemcpyAsync(h, nb, (size_t)2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (info_out)
    for (int k = 0; k < nrhs; ++k) {
      const double rel = h[k] > 0.0 ? std::sqrt(h[nrhs + k] / h[k]) : 0.0;
      info_out[k] = {refine, 1, rel};
    }
}

// ================================================================== PCG ====
// Preconditioned conjugate gradients with M = the factor (Sec. 3: the
// preconditioner serves any Krylov solver, CG among them), every
// right-hand side its own coefficients.  x0 = 0; flexible beta
// <z_new, r_new - r_old> / <z_old, r_old> (the FP32 apply is not an exactly
// fixed linear operator); a column stops when its recursive residual meets
// tol or it reaches maxit iterations, then every column's true residual
// b - A x is formed and columns that miss tol start again from x.  One host
// read of the residual norms per iteration.
void NumericBase::pcg(int nrhs, const double* b, double* x, double tol, int maxit, hipStream_t st,
                      mf_gmres_info* info_out, mf_status* st_out) {
  const int N = sym->n;
  const int64_t vs = (int64_t)N * nrhs;
  g_V.ensure((size_t)2 * vs * 8, &ms, st);
  g_Z.ensure((size_t)3 * vs * 8, &ms, st);
  g_small.ensure((size_t)7 * nrhs * 8 + (size_t)nrhs * 4, &ms, st);
  g_partial.ensure((size_t)mdot_chunks(nrhs) * 2 * nrhs * 8, &ms, st);
  double* r = g_V.as<double>();
  double* rprev = r + vs;                 // right after r: one mdot takes both
  double* z = g_Z.as<double>();
  double* p = z + vs;
  double* q = p + vs;
  double* sm = g_small.as<double>();
  double* S[2] = {sm, sm + 2 * nrhs};     // per iteration: <r, z> (first nrhs), <r_old, z> (next nrhs)
  double* pq = sm + 4 * nrhs;
  double* rr = pq + nrhs;
  double* bn = rr + nrhs;
  int* act = reinterpret_cast<int*>(bn + nrhs);
  double* part = g_partial.as<double>();
  PinnedScratch pin((size_t)nrhs * (sizeof(double) + sizeof(int)), st);
  double* hr = pin.as<double>(0);
  int* hact = pin.as<int>((size_t)nrhs * sizeof(double));
  auto read = [&](const double* d) {
    HIPCHK(hipMemcpyAsync(hr, d, (size_t)nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  };
  auto upload_act = [&]() {
    HIPCHK(hipMemcpyAsync(act, hact, (size_t)nrhs * sizeof(int), hipMemcpyHostToDevice, st));
  };
  launch_mdot(b, 0, 1, b, N, nrhs, part, bn, 0, st);
  read(bn);
  std::vector<double> bnorm(nrhs), relres(nrhs, 0.0);
  std::vector<int> iters(nrhs, 0), conv(nrhs, 0);
  for (int k = 0; k < nrhs; ++k) {
    bnorm[k] = std::sqrt(hr[k]);
    conv[k] = bnorm[k] == 0.0;
  }
  launch_fill<double>(x, vs, 0.0, st);
  launch_axpby(b, b, r, 1.0, 0.0, vs, st);   // r = b
  for (;;) {
    bool any = false;
    for (int k = 0; k < nrhs; ++k) {
      hact[k] = !conv[k] && iters[k] < maxit;
      any |= hact[k] != 0;
    }
    if (!any) break;
    upload_act();
    // (re)start every active column from x with its residual r
    apply(nrhs, r, z, st);
    launch_axpby(z, z, p, 1.0, 0.0, vs, st);                 // p = z
    launch_mdot(r, 0, 1, z, N, nrhs, part, S[0], 0, st);     // <r, z>
    int cur = 0;
    for (;;) {
      spmv(nrhs, p, q, 1.0, 0.0, st);
      launch_mdot(p, 0, 1, q, N, nrhs, part, pq, 0, st);
      launch_cg_xr(x, r, rprev, p, q, S[cur], pq, act, N, nrhs, st);
      launch_mdot(r, 0, 1, r, N, nrhs, part, rr, 0, st);
      read(rr);
      any = false;
      for (int k = 0; k < nrhs; ++k) {
        if (!hact[k]) continue;
        ++iters[k];
        if (std::sqrt(hr[k]) <= tol * bnorm[k] || iters[k] >= maxit) hact[k] = 0;
        any |= hact[k] != 0;
      }
      if (!any) break;
      upload_act();
      apply(nrhs, r, z, st);
      launch_mdot(r, vs, 2, z, N, nrhs, part, S[1 - cur], 0, st);   // <r, z>, <r_old, z>
      launch_cg_p(p, z, S[1 - cur], S[1 - cur] + nrhs, S[cur], act, N, nrhs, st);
      cur = 1 - cur;
    }
    // true residuals
    spmv(nrhs, x, q, 1.0, 0.0, st);
    launch_axpby(b, q, r, 1.0, -1.0, vs, st);
    launch_mdot(r, 0, 1, r, N, nrhs, part, rr, 0, st);
    read(rr);
    for (int k = 0; k < nrhs; ++k) {
      relres[k] = bnorm[k] > 0.0 ? std::sqrt(hr[k]) / bnorm[k] : 0.0;
      if (relres[k] <= tol) conv[k] = 1;
    }
  }
  bool ok = true;
  for (int k = 0; k < nrhs; ++k) {
    ok &= conv[k] != 0;
    if (info_out) info_out[k] = {iters[k], conv[k], relres[k]};
  }
  *st_out = ok ? MF_OK : MF_ENOCONV;
}

// Device bytes of a factorisation before it runs.  Exact for the front
// workspace, the dense fronts and the fixed buffers; the HODLR part assumes
// every block rank r <= min(rows, cols, rank_cap, 8 sqrt(max(rows, cols)))
// (ranks grow like sqrt(n), Sec. 1).  persistent = what a resident handle
// holds with apply and GMRES(restart) workspaces for nrhs right-hand sides;
// peak = the most held during mf_factor.
void estimate_bytes(const Symbolic& s, const mf_opts& o, int nrhs, int restart, int64_t& persistent,
                    int64_t& peak) {
  const double es = o.precision == MF_FP64 ? 8.0 : 4.0;
  const double eb = (o.precision == MF_FP32 && o.uv_bf16) ? 2.0 : es;   // stored bases U, V, W
  const bool hodlr = o.method == MF_METHOD_HODLR;
  const bool sampled = hodlr && o.sampled != 0;
  std::vector<int64_t> ro, re, fo;
  std::vector<char> staged(s.fronts.size(), 1);
  if (sampled)
    for (size_t p = 0; p < s.fronts.size(); ++p) staged[p] = s.fronts[p].n() < o.n_c;
  const double ws = (double)workspace_plan(s, ro, re, fo, &staged) * es;
  // sampled: a level's gathered samples, and the compressed updates kept for
  // the parents (ff leaf blocks, ff bases, W S) while the next level runs
  std::vector<double> lvl_samples(s.levels.size(), 0.0), lvl_kept(s.levels.size(), 0.0);
  const double csr = 12.0 * s.nnz + 4.0 * (s.n + 1) + 8.0 * s.n;
  double fac = 0, scratch = 0, apply = 0;
  std::vector<double> lvl_scratch(s.levels.size(), 0.0);
  for (const Front& f : s.fronts) {
    const double np = f.npiv, nf = f.nf();
    apply += (f.n() + np) * nrhs * es;
    if (!hodlr || f.n() < o.n_c) {
      fac += (np * np + nf * np) * es;
      continue;
    }
    auto rk = [&](const Block& B) {
      const double r = std::min({(double)B.nr, (double)B.nc, (double)o.rank_cap,
                                 std::ceil(8.0 * std::sqrt((double)std::max(B.nr, B.nc)))});
      return r;
    };
    double w = 0, rtop = 0;
    for (const Block& B : f.blocks) {
      const double r = rk(B);
      if (B.kind == 0) rtop = r;
      if (B.kind == 1) {
        fac += (B.nr + B.nc) * r * eb + 4.0 * r * r * es;   // U, V and the capacitance inverse
        w += r;
        apply += 4.0 * r * nrhs * es;
      }
      lvl_scratch[f.height] += (B.nr + B.nc) * std::min((double)o.rank_cap, (double)std::min(B.nr, B.nc)) * es;
      if (sampled) {
        const double cap = o.bdlr_cap > 0 ? o.bdlr_cap : (es == 8.0 ? 128.0 : 192.0);   // BDLR set bound
        const double nI = std::min((double)B.nr, cap), nJ = std::min((double)B.nc, cap);
        const bool full = B.nr <= 256 && B.nc <= 256;
        lvl_samples[f.height] += (full ? (double)B.nr * B.nc : B.nr * nJ + nI * B.nc + nI * nJ) * es;
        if (B.kind == 2) lvl_kept[f.height] += (B.nr + B.nc) * r * es;
        if (B.kind == 0) lvl_kept[f.height] += B.nr * r * es;
      }
    }
    for (const TreeNode& t : f.pp_tree)
      if (t.left < 0) {
        fac += (double)t.size * t.size * es;                  // leaf inverses
        if (sampled) lvl_samples[f.height] += (double)t.size * t.size * es;
      }
    if (sampled)
      for (const TreeNode& t : f.ff_tree)
        if (t.left < 0) lvl_kept[f.height] += (double)t.size * t.size * es;
    fac += np * (rtop + w) * es + nf * rtop * eb;             // G (X and the SMW columns), W
    apply += rtop * nrhs * es;
  }
  for (double v : lvl_scratch) scratch = std::max(scratch, v);
  double samples = 0;
  for (size_t h = 0; h < s.levels.size(); ++h)
    samples = std::max(samples, lvl_samples[h] + lvl_kept[h] + (h > 0 ? lvl_kept[h - 1] : 0.0));
  const double gm = 8.0 * s.n * nrhs * (2.0 * restart + 3.0);
  const double fixed = (double)kSplitFactorBytes + (64 << 20);   // split-K partials, one descriptor chunk
  persistent = (int64_t)(fac + csr + apply + gm + kSplitPlanBytes);
  peak = (int64_t)(ws + fac + csr + scratch + samples + fixed + 16.0 * s.nnz);
}

void set_phase2_wait_ticks(long long ticks) { g_phase2_wait_override.store(ticks); }
void set_record_block_errors(bool on) { g_record_block_errors.store(on); }

std::unique_ptr<NumericBase> make_numeric(const Symbolic& s, const double* vals, const mf_opts& o) {
  if (o.precision == MF_FP64) return std::make_unique<Numeric<double>>(s, vals, o);
  return std::make_unique<Numeric<float>>(s, vals, o);
}

}  // namespace mfh
