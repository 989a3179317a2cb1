// Optional per-kernel timing: HIP events recorded on the launch stream
// around each launch of the selected kernels, with the launch's algorithmic
// work (flops, bytes) as counted on the host.  Off unless started through
// mf_prof_start; then each timed launch costs two event records.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace mfh {

// Each kind is one device kernel (one name in a kernel trace); float64 and
// float32 instantiations are separate kinds, float64 first.
enum ProfKind : int {
  PK_GEMM_F64, PK_GEMM_F32,
  PK_GEMMN_F64, PK_GEMMN_F32,          // 64 x 16 tiles (right-hand-side blocks)
  PK_GEMM_REDUCE_F64, PK_GEMM_REDUCE_F32,
  PK_GEMMNF_F64, PK_GEMMNF_F32,        // 64 x 16 tiles reading folded split-K partials
  PK_POTRF64_F64, PK_POTRF64_F32,      // leaf size <= 64
  PK_POTRF128_F64, PK_POTRF128_F32,
  PK_SKREG_FULL_F64, PK_SKREG_FULL_F32,
  PK_SKREG_HAT_F64, PK_SKREG_HAT_F32,
  PK_SKELFAC_F64, PK_SKELFAC_F32,
  PK_PHASE2_F64, PK_PHASE2_F32,
  PK_PHASE2CL_F64, PK_PHASE2CL_F32,    // multi-workgroup phase 2, slices in LDS
  PK_PHASE2CG_F64, PK_PHASE2CG_F32,    // multi-workgroup phase 2, in place
  PK_EXTADD_F64, PK_EXTADD_F32,
  PK_GJ64, PK_GJ128, PK_GJ192, PK_GJWIDE,   // capacitance inverse by matrix size
  PK_SPMV,
  PK_COUNT
};

template <typename T>
constexpr int pk(int f64_kind) { return sizeof(T) == 4 ? f64_kind + 1 : f64_kind; }

const char* prof_name(int kind);
// true while a timing session selects this kernel kind
bool prof_selected(int kind);
// while set on this thread, no launch is timed (used while a HIP graph is
// recorded: its nodes are replayed untimed)
void prof_suspend(bool on);

// id >= 0 when the launch is timed; -1 otherwise (all calls then do nothing).
// A timed record hands its two events to the next kernel launched by this
// thread through MFH_LAUNCH, which has the runtime stamp the kernel's own
// start and end (no launch gap inside the interval).  For a launch API that
// cannot take events, prof_stream_start records the start on the stream and
// prof_end the end; a record that no launch used is dropped.
int prof_begin(int kind, hipStream_t st, double flops, double bytes);
void prof_end(int id, hipStream_t st);
bool prof_take(hipEvent_t* start, hipEvent_t* stop);
// for a launch that cannot take events: record the start on the stream now
void prof_stream_start(int id, hipStream_t st);

// launch through here so that a pending timing record gets kernel-stamped events
#define MFH_LAUNCH(kernel, grid, block, shmem, stream, ...)                                         \
  do {                                                                                              \
    hipEvent_t mfh_a_, mfh_b_;                                                                      \
    if (::mfh::prof_take(&mfh_a_, &mfh_b_))                                                         \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, mfh_a_, mfh_b_, 0, __VA_ARGS__);    \
    else                                                                                            \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                          \
  } while (0)
// work known only after the launch (e.g. ranks read back later)
void prof_add(int id, double flops, double bytes);

struct ProfTotal {
  int kind;
  int64_t launches;
  double seconds, flops, bytes;
};
// names: semicolon-separated kernel names to time; empty = every kind
void prof_start(const std::string& names);
// waits for the recorded events, returns per-kind totals, stops timing
std::vector<ProfTotal> prof_stop();

}  // namespace mfh
