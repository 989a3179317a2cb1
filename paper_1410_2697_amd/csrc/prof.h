// Optional per-kernel timing: HIP events recorded on the launch stream
// around each launch of the selected kernels, with the launch's algorithmic
// work (flops, bytes) as counted on the host.  Off unless started through
// mf_prof_start; then each timed launch costs two event records.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace mfh {

// Each kind is one device kernel (one name in a kernel trace); float64 and
// float32 instantiations are separate kinds, float64 first.
enum ProfKind : int {
  PK_GEMM_F64, PK_GEMM_F32,
  PK_GEMM_REDUCE_F64, PK_GEMM_REDUCE_F32,
  PK_POTRF64_F64, PK_POTRF64_F32,      // leaf size <= 64
  PK_POTRF128_F64, PK_POTRF128_F32,
  PK_SKREG_FULL_F64, PK_SKREG_FULL_F32,
  PK_SKREG_HAT_F64, PK_SKREG_HAT_F32,
  PK_SKELFAC_F64, PK_SKELFAC_F32,
  PK_PHASE2_F64, PK_PHASE2_F32,
  PK_PHASE2C_F64, PK_PHASE2C_F32,
  PK_EXTADD_F64, PK_EXTADD_F32,
  PK_GJ,
  PK_SPMV,
  PK_COUNT
};

template <typename T>
constexpr int pk(int f64_kind) { return sizeof(T) == 4 ? f64_kind + 1 : f64_kind; }

const char* prof_name(int kind);

// id >= 0 when the launch is timed; -1 otherwise (all calls then do nothing)
int prof_begin(int kind, hipStream_t st, double flops, double bytes);
void prof_end(int id, hipStream_t st);
// work known only after the launch (e.g. ranks read back later)
void prof_add(int id, double flops, double bytes);

struct ProfTotal {
  int kind;
  int64_t launches;
  double seconds, flops, bytes;
};
// names: comma-separated kernel names to time; empty = every kind
void prof_start(const std::string& names);
// waits for the recorded events, returns per-kind totals, stops timing
std::vector<ProfTotal> prof_stop();

}  // namespace mfh
