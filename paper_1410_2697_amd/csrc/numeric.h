// Numeric factor, preconditioner apply and GMRES driver (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/mfh.h"
#include "kernels.h"
#include "symbolic.h"

namespace mfh {

struct Err {
  mf_status code;
  std::string msg;
};

// Device memory accounting shared by all allocations of one factor.
struct MemStats {
  int64_t current = 0, peak = 0;
  void add(int64_t b) { current += b; if (current > peak) peak = current; }
  void sub(int64_t b) { current -= b; }
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  MemStats* ms = nullptr;
  int dev = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release();
  void alloc(size_t b, MemStats* m);        // throws Err on failure
  void ensure(size_t b, MemStats* m, hipStream_t st);   // grows (synchronising) when needed
  // grows without synchronising: the old block moves to `retired`, whose
  // owner releases it after the stream work that may use it has finished
  void grow(size_t b, MemStats* m, std::vector<std::unique_ptr<DevBuf>>& retired);
  // grows to exactly b bytes after synchronising the stream and releasing
  // the old block and `retired`, so that the high-water mark never holds a
  // dead block beside its successor (for the largest per-level scratch)
  void regrow(size_t b, MemStats* m, hipStream_t st, std::vector<std::unique_ptr<DevBuf>>& retired);
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Bump allocator over device chunks for the persistent factor arrays.
struct Arena {
  std::vector<std::unique_ptr<DevBuf>> chunks;
  size_t off = 0;
  int64_t used = 0;
  MemStats* ms = nullptr;
  void* alloc(size_t bytes);
  template <typename T> T* alloc_n(int64_t n) { return static_cast<T*>(alloc((size_t)std::max<int64_t>(n, 1) * sizeof(T))); }
};

// Host blob of descriptor arrays uploaded in one copy.
struct Blob {
  std::vector<char> h;
  template <typename D>
  size_t add(const std::vector<D>& v) {
    size_t o = (h.size() + 255) & ~size_t(255);
    h.resize(o + v.size() * sizeof(D));
    if (!v.empty()) memcpy(h.data() + o, v.data(), v.size() * sizeof(D));
    return o;
  }
};

// throws Err{MF_EHIP} when a HIP call fails
#define HIPCHK(x)                                                                              \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) throw Err{MF_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

class NumericBase {
 public:
  virtual ~NumericBase() = default;
  virtual void apply(int nrhs, const double* r, double* z, hipStream_t st) = 0;
  // the same apply with no device allocation (mf_apply_noalloc)
  virtual void apply_noalloc(int nrhs, const double* r, double* z, hipStream_t st) = 0;
  void spmv(int nrhs, const double* x, double* y, double alpha, double beta, hipStream_t st,
            const int* win = nullptr);
  // win: host int32[2 * nrhs] row windows of the columns (independent systems
  // solved together, each column zero outside its system's rows), or null
  void gmres(int nrhs, const double* b, double* x, double tol, const mf_gmres_opts& o, mf_gmres_info* info,
             mf_status* st_out, const int32_t* win = nullptr);
  void pcg(int nrhs, const double* b, double* x, double tol, int maxit, hipStream_t st, mf_gmres_info* info,
           mf_status* st_out);
  void direct_solve(int nrhs, const double* b, double* x, int refine, hipStream_t st, mf_gmres_info* info);
  mf_factor_info info{};
  // per compressed block, when recording is on (set_record_block_errors):
  // front, block, rank, max|B|, |u_11|, max|B - U V^T| (float64, before any
  // bfloat16 rounding of the bases)
  struct BlockErr { int front, block, rank; double bmax, u11, emax; };
  std::vector<BlockErr> block_errors;
  uint64_t uid = 0;              // process-unique handle number (never reused)
  std::vector<int> ranks;        // per global block, -1 for dense fronts
  const Symbolic* sym = nullptr;
  mf_opts opts{};
  MemStats ms;
  int device = 0;
  // device copy of A (original order) and permutations
  DevBuf d_rowptr, d_colind, d_vals, d_perm, d_iperm, d_status;
  // GMRES workspace
  DevBuf g_V, g_Z, g_w, g_r, g_small, g_partial;
  // Streams this handle has launched work on, each with an event recorded
  // after its latest work.  Before the handle's device blocks go back to the
  // allocator cache it waits for these events (not for the whole device,
  // which may be running other handles' work).
  void note_stream(hipStream_t st);
  void wait_streams();
  std::mutex ev_mu;
  std::vector<std::pair<hipStream_t, hipEvent_t>> stream_events;
};

std::unique_ptr<NumericBase> make_numeric(const Symbolic& s, const double* vals, const mf_opts& o);
// Barrier wait of the multi-workgroup phase 2, in ticks of the device's
// constant-rate clock: 0 restores the default (two seconds), < 0 makes every
// workgroup give up at its first barrier (test hook for the error path).
void set_phase2_wait_ticks(long long ticks);
// Test hook: factorisations started while on keep a float64 copy of every
// block before compression and record its truncation error (block_errors);
// assembled fronts only (a sampled front never forms its blocks).
void set_record_block_errors(bool on);
// message of the MF_EHIP a phase-2 barrier give-up ends the factorisation with
constexpr const char* kPhase2WaitMsg = "phase-2 workgroups did not meet at their barrier";
// Front workspace plan (elements): the staged fronts of one level share a
// region that lives until the level of its last parent is done; regions are
// placed first fit over offsets.  `staged` (null: every front) marks the
// fronts that take dense staging.  Returns the peak.
int64_t workspace_plan(const Symbolic& s, std::vector<int64_t>& reg_off, std::vector<int64_t>& reg_elems,
                       std::vector<int64_t>& front_elem_off, const std::vector<char>* staged = nullptr);
void estimate_bytes(const Symbolic& s, const mf_opts& o, int nrhs, int restart, int64_t& persistent,
                    int64_t& peak);

}  // namespace mfh
