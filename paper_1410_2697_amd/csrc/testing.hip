// Kernel-level test hooks (include/mfh_testing.h): one problem per call,
// synchronous, on the null stream.
#include <algorithm>
#include <string>

#include "../../include/mfh_testing.h"
#include "kernels.h"
#include "numeric.h"

namespace {
thread_local std::string t_err;

mf_status hip_ok(hipError_t e) {
  if (e == hipSuccess) return MF_OK;
  t_err = hipGetErrorString(e);
  return MF_EHIP;
}

template <typename T>
mf_status gemm_t(int m, int n, int k, const void* A, int lda, int opA, const void* B, int ldb, int opB, void* C,
                 int ldc, double alpha, double beta, int flags, int kchunk, const int* arow = nullptr,
                 const int* brow = nullptr, const mfh::FoldDesc<T>* fold = nullptr) {
  mfh::GemmDesc<T> d{};
  d.A = static_cast<const T*>(A); d.B = static_cast<const T*>(B); d.C = static_cast<T*>(C);
  d.arow = arow; d.brow = brow;
  d.m = m; d.n = n; d.k = k; d.lda = lda; d.ldb = ldb; d.ldc = ldc; d.opA = opA; d.opB = opB;
  d.flags = flags; d.alpha = alpha; d.beta = beta;
  // at most 16 columns: the 64 x 16 tile variant (the reduction walks 64 x 64 tiles)
  const int tn = n <= mfh::kTileNarrow ? mfh::kTileNarrow : mfh::kTile;
  d.tiles_m = (m + mfh::kTile - 1) / mfh::kTile;
  d.tiles_n = (n + tn - 1) / tn;
  d.tile0 = 0;
  d.ksplit = 1;
  if (kchunk > 0 && k > 0) {
    d.ksplit = (k + kchunk - 1) / kchunk;
    d.kchunk = kchunk;
  }
  const int otiles = d.tiles_m * d.tiles_n;
  if (otiles == 0) return MF_OK;
  mfh::GemmDesc<T>* dd = nullptr;
  mf_status s = hip_ok(hipMalloc(&dd, 2 * sizeof(d) + sizeof(mfh::FoldDesc<T>)));
  if (s != MF_OK) return s;
  auto* df = reinterpret_cast<mfh::FoldDesc<T>*>(dd + 2);
  if (d.ksplit > 1) {
    s = hip_ok(hipMalloc(&d.part, (size_t)d.ksplit * m * n * sizeof(T)));
    if (s != MF_OK) { hipFree(dd); return s; }
  }
  mfh::GemmDesc<T> r = d;
  r.tiles_n = (n + mfh::kTile - 1) / mfh::kTile;
  hipMemcpy(dd, &d, sizeof(d), hipMemcpyHostToDevice);
  hipMemcpy(dd + 1, &r, sizeof(r), hipMemcpyHostToDevice);
  if (fold) {
    hipMemcpy(df, fold, sizeof(*fold), hipMemcpyHostToDevice);
    mfh::launch_gemm_fold<T>(dd, df, 1, otiles * d.ksplit, nullptr);
  } else {
    mfh::launch_gemm<T>(dd, 1, otiles * d.ksplit, nullptr, tn);
  }
  if (d.ksplit > 1) mfh::launch_gemm_reduce<T>(dd + 1, 1, r.tiles_m * r.tiles_n, nullptr);
  s = hip_ok(hipDeviceSynchronize());
  hipFree(dd);
  if (d.part) hipFree(d.part);
  return s;
}

template <typename T>
mf_status potrf_t(int n, void* A, int lda, void* Inv, int ldi, int* status_out) {
  mfh::PotrfDesc<T> d{};
  d.A = static_cast<T*>(A); d.lda = lda; d.n = n; d.Inv = static_cast<T*>(Inv); d.ldi = ldi;
  mfh::PotrfDesc<T>* dd = nullptr;
  int* st = nullptr;
  mf_status s = hip_ok(hipMalloc(&dd, sizeof(d)));
  if (s == MF_OK) s = hip_ok(hipMalloc(&st, sizeof(int)));
  if (s != MF_OK) return s;
  hipMemcpy(dd, &d, sizeof(d), hipMemcpyHostToDevice);
  hipMemset(st, 0, sizeof(int));
  mfh::launch_potrf<T>(dd, 1, n, st, nullptr);
  s = hip_ok(hipDeviceSynchronize());
  if (s == MF_OK && status_out) hipMemcpy(status_out, st, sizeof(int), hipMemcpyDeviceToHost);
  hipFree(dd);
  hipFree(st);
  return s;
}

template <typename T>
mf_status skel_t(void* F, int ld, int r0, int nr, int c0, int nc, const int* I, int nI, const int* J, int nJ,
                 double eps, int adaptive, int cap, void* U, void* V, int* rank_out) {
  const int kcap = nI < nJ ? nI : nJ;
  const bool full = nr <= mfh::skreg_full_rows<T>() && nc <= mfh::skreg_full_cols<T>();
  char* scratch = nullptr;
  const size_t bytes = 4096 + (size_t)(kcap + 1) * (kcap + 1) * sizeof(T) + 8 * (size_t)(cap + 1) + 1024;
  mf_status s = hip_ok(hipMalloc(&scratch, bytes));
  if (s != MF_OK) return s;
  int* rank1 = reinterpret_cast<int*>(scratch);
  int* rank = rank1 + 1;
  int* status = rank1 + 2;
  double* u11 = reinterpret_cast<double*>(scratch + 64);
  T* M = reinterpret_cast<T*>(scratch + 128);
  int* pr = reinterpret_cast<int*>(scratch + 128 + (size_t)(kcap + 1) * (kcap + 1) * sizeof(T));
  int* pc = pr + cap + 1;
  hipMemset(scratch, 0, 128);
  mfh::SkRegDesc<T> sd{};
  sd.F = static_cast<T*>(F); sd.ld = ld; sd.r0 = r0; sd.nr = nr; sd.c0 = c0; sd.nc = nc;
  sd.I = I; sd.nI = nI; sd.J = J; sd.nJ = nJ; sd.piv_r = pr; sd.piv_c = pc;
  sd.rank1 = rank1; sd.rank = rank; sd.u11 = u11; sd.cap = cap;
  sd.U = static_cast<T*>(U); sd.ldu = nr; sd.V = static_cast<T*>(V); sd.ldv = nc;
  sd.M = M; sd.ldm = kcap > 0 ? kcap : 1;
  mfh::SkelFacDesc<T> fd{};
  fd.F = static_cast<T*>(F); fd.ld = ld; fd.FR = fd.F; fd.ldr = ld; fd.r0 = r0; fd.nr = nr; fd.c0 = c0; fd.nc = nc;
  fd.piv_r = pr; fd.piv_c = pc; fd.M = M; fd.ldm = sd.ldm; fd.rank = rank1;
  fd.U = static_cast<T*>(U); fd.ldu = nr; fd.V = static_cast<T*>(V); fd.ldv = nc;
  fd.wgU = (nr + mfh::kSkelFacRows - 1) / mfh::kSkelFacRows; fd.wg0 = 0;
  const int wgs = fd.wgU + (nc + mfh::kSkelFacRows - 1) / mfh::kSkelFacRows;
  mfh::GemmDesc<T> gdsc{};
  gdsc.A = fd.U; gdsc.lda = nr; gdsc.B = fd.V; gdsc.ldb = nc; gdsc.opB = 1;
  gdsc.C = static_cast<T*>(F) + r0 + (size_t)c0 * ld; gdsc.ldc = ld;
  gdsc.m = nr; gdsc.n = nc; gdsc.k = kcap; gdsc.kdev = rank1; gdsc.alpha = -1.0; gdsc.beta = 1.0;
  gdsc.tiles_m = (nr + 63) / 64;
  gdsc.tiles_n = (nc + 63) / 64;
  gdsc.ksplit = 1;
  const int gtiles = gdsc.tiles_m * gdsc.tiles_n;
  mfh::Phase2Desc<T> pd{};
  pd.F = static_cast<T*>(F); pd.ld = ld; pd.r0 = r0; pd.nr = nr; pd.c0 = c0; pd.nc = nc;
  pd.piv_r = pr; pd.piv_c = pc; pd.rank1 = rank1; pd.u11 = u11; pd.U = fd.U; pd.ldu = nr; pd.V = fd.V;
  pd.ldv = nc; pd.cap = cap; pd.rank = rank;
  char* dd = nullptr;
  s = hip_ok(hipMalloc(&dd, 4096));
  if (s != MF_OK) { hipFree(scratch); return s; }
  hipMemcpy(dd, &sd, sizeof(sd), hipMemcpyHostToDevice);
  hipMemcpy(dd + 1024, &fd, sizeof(fd), hipMemcpyHostToDevice);
  hipMemcpy(dd + 2048, &gdsc, sizeof(gdsc), hipMemcpyHostToDevice);
  hipMemcpy(dd + 3072, &pd, sizeof(pd), hipMemcpyHostToDevice);
  if (full) {
    mfh::launch_skreg_full<T>(reinterpret_cast<mfh::SkRegDesc<T>*>(dd), 1, eps, adaptive ? 1 : 0, status, nullptr);
  } else {
    mfh::launch_skreg_hat<T>(reinterpret_cast<mfh::SkRegDesc<T>*>(dd), 1, eps, status, nullptr);
    mfh::launch_skelfac<T>(reinterpret_cast<mfh::SkelFacDesc<T>*>(dd + 1024), 1, wgs, kcap > 0 ? kcap : 1, nullptr);
    if (adaptive) {
      mfh::launch_gemm<T>(reinterpret_cast<mfh::GemmDesc<T>*>(dd + 2048), 1, gtiles, nullptr);
      // 1: slices in LDS; 3: slices updated in place; 2: one workgroup
      const bool slds = adaptive == 1;
      int wc = adaptive == 1 ? mfh::phase2_coop_wcols<T>(nr) : (adaptive == 3 ? 4 : 0);
      int nwg = wc > 0 && nr <= mfh::kPhase2CoopMaxRows ? (nc + wc - 1) / wc : 0;
      const size_t lds = slds ? (size_t)mfh::kPhase2CoopLds : mfh::phase2_coop_lds<T>(nr, wc, false);
      if (nwg > mfh::phase2_coop_capacity<T>(lds, slds)) nwg = 0;
      if (nwg > 0) {
        char* cs = nullptr;   // tagged key slots, candidate columns
        const size_t kb = 256 + (size_t)2 * nwg * 8, cb = (size_t)2 * nwg * nr * sizeof(T);
        s = hip_ok(hipMalloc(&cs, kb + cb));
        if (s == MF_OK) {
          mfh::launch_fill<unsigned long long>(reinterpret_cast<unsigned long long*>(cs + 256), 2 * nwg, 1ull << 63,
                                               nullptr);
          mfh::Phase2CoopDesc<T> qd{};
          qd.F = pd.F; qd.ld = ld; qd.r0 = r0; qd.nr = nr; qd.c0 = c0; qd.nc = nc;
          qd.piv_r = pr; qd.piv_c = pc; qd.rank1 = rank1; qd.u11 = u11; qd.U = pd.U; qd.ldu = nr; qd.V = pd.V;
          qd.ldv = nc; qd.cap = cap; qd.rank = rank;
          qd.keys = reinterpret_cast<unsigned long long*>(cs + 256);
          qd.cand = reinterpret_cast<T*>(cs + kb);
          qd.wg0 = 0; qd.nwg = nwg; qd.wcols = (nc + nwg - 1) / nwg;
          hipMemcpy(dd + 3072, &qd, sizeof(qd), hipMemcpyHostToDevice);
          s = hip_ok(mfh::launch_phase2_coop<T>(reinterpret_cast<mfh::Phase2CoopDesc<T>*>(dd + 3072), 1, nwg, lds,
                                                slds, eps, status, 200000000LL, nullptr));
          if (s == MF_OK) s = hip_ok(hipDeviceSynchronize());
          hipFree(cs);
        }
        if (s != MF_OK) { hipFree(dd); hipFree(scratch); return s; }
      } else {
        mfh::launch_phase2<T>(reinterpret_cast<mfh::Phase2Desc<T>*>(dd + 3072), 1, nr + nc, eps, status, nullptr);
      }
    }
  }
  s = hip_ok(hipDeviceSynchronize());
  int stat = 0;
  if (s == MF_OK) {
    hipMemcpy(rank_out, rank, sizeof(int), hipMemcpyDeviceToHost);
    hipMemcpy(&stat, status, sizeof(int), hipMemcpyDeviceToHost);
  }
  hipFree(dd);
  hipFree(scratch);
  if (s == MF_OK && (stat & 8)) {
    t_err = "phase-2 workgroups did not meet at their barrier";
    return MF_EHIP;
  }
  if (s == MF_OK && (stat & 16)) {
    t_err = "a pivot was not finite";
    return MF_ENOTSPD;
  }
  return s;
}
}  // namespace

extern "C" {

mf_status mfh_test_mfma_layout(int32_t precision, int32_t* rows, int32_t* cols, int32_t* assumed) {
  if (!rows || !cols || !assumed) return MF_EINVAL;
  int* d = nullptr;
  mf_status s = hip_ok(hipMalloc(&d, 3 * 256 * sizeof(int)));
  if (s != MF_OK) return s;
  if (precision == MF_FP64) mfh::launch_mfma_probe<double>(d, d + 256, d + 512, nullptr);
  else mfh::launch_mfma_probe<float>(d, d + 256, d + 512, nullptr);
  s = hip_ok(hipDeviceSynchronize());
  if (s == MF_OK) {
    hipMemcpy(rows, d, 256 * sizeof(int), hipMemcpyDeviceToHost);
    hipMemcpy(cols, d + 256, 256 * sizeof(int), hipMemcpyDeviceToHost);
    hipMemcpy(assumed, d + 512, 256 * sizeof(int), hipMemcpyDeviceToHost);
  }
  hipFree(d);
  return s;
}

mf_status mfh_test_gemm(int32_t precision, int32_t m, int32_t n, int32_t k, const void* A, int32_t lda, int32_t opA,
                        const void* B, int32_t ldb, int32_t opB, void* C, int32_t ldc, double alpha, double beta,
                        int32_t flags, int32_t kchunk) {
  if (m < 0 || n < 0 || k < 0 || !C || kchunk < 0 || kchunk % mfh::kGemmSplitAlign != 0) return MF_EINVAL;
  if (precision == MF_FP64)
    return gemm_t<double>(m, n, k, A, lda, opA, B, ldb, opB, C, ldc, alpha, beta, flags, kchunk);
  return gemm_t<float>(m, n, k, A, lda, opA, B, ldb, opB, C, ldc, alpha, beta, flags, kchunk);
}

mf_status mfh_test_gemm_rows(int32_t precision, int32_t m, int32_t n, int32_t k, const void* A, int32_t lda,
                             int32_t opA, const int32_t* arow, const void* B, int32_t ldb, int32_t opB,
                             const int32_t* brow, void* C, int32_t ldc, double alpha, double beta, int32_t kchunk) {
  if (m < 0 || n < 0 || k < 0 || !C || kchunk < 0 || kchunk % mfh::kGemmSplitAlign != 0) return MF_EINVAL;
  if (precision == MF_FP64)
    return gemm_t<double>(m, n, k, A, lda, opA, B, ldb, opB, C, ldc, alpha, beta, 0, kchunk, arow, brow);
  return gemm_t<float>(m, n, k, A, lda, opA, B, ldb, opB, C, ldc, alpha, beta, 0, kchunk, arow, brow);
}

mf_status mfh_test_gemm_fold(int32_t precision, int32_t m, int32_t n, int32_t k, const void* A, int32_t lda,
                             int32_t opA, const void* B, int32_t ldb, void* C, int32_t ldc, double alpha,
                             double beta, int32_t kchunk, int32_t bsplit, const void* part0, const void* part1,
                             const int32_t* slices, const int32_t* ld, const double* coef) {
  if (m < 0 || n < 0 || n > mfh::kTileNarrow || k < 0 || !C || kchunk < 0 || kchunk % mfh::kGemmSplitAlign != 0 ||
      bsplit < 0 || bsplit > k || !slices || !ld || !coef)
    return MF_EINVAL;
  const void* parts[2] = {part0, part1};
  const int rows[2] = {bsplit, k - bsplit};
  for (int s = 0; s < 2; ++s)
    if (slices[s] < 0 || slices[s] > mfh::kFoldSlices ||
        (slices[s] > 0 && (!parts[s] || ld[s] < std::max(rows[s], 1))))
      return MF_EINVAL;
  auto run = [&](auto zero) -> mf_status {
    using T = decltype(zero);
    mfh::FoldDesc<T> f{};
    f.split = bsplit;
    for (int s = 0; s < 2; ++s) {
      f.part[s] = slices[s] > 0 ? static_cast<const T*>(parts[s]) : nullptr;
      f.slices[s] = slices[s];
      f.ld[s] = ld[s];
      f.alpha[s] = coef[2 * s];
      f.beta[s] = coef[2 * s + 1];
    }
    return gemm_t<T>(m, n, k, A, lda, opA, B, ldb, 0, C, ldc, alpha, beta, 0, kchunk, nullptr, nullptr, &f);
  };
  return precision == MF_FP64 ? run(0.0) : run(0.0f);
}

mf_status mfh_test_potrf(int32_t precision, int32_t n, void* A, int32_t lda, void* Inv, int32_t ldi,
                         int32_t* status_out) {
  if (n < 1 || n > 128 || !A) return MF_EINVAL;
  if (precision == MF_FP64) return potrf_t<double>(n, A, lda, Inv, ldi, status_out);
  return potrf_t<float>(n, A, lda, Inv, ldi, status_out);
}

mf_status mfh_test_inverse(int32_t n, double* A, int32_t lda, int32_t* status_out) {
  if (n < 1 || n > mfh::kInvMax || lda < n || !A) return MF_EINVAL;
  mfh::InvDesc d{};
  d.A = A; d.n = n; d.ld = lda;
  mfh::InvDesc* dd = nullptr;
  int* st = nullptr;
  mf_status s = hip_ok(hipMalloc(&dd, sizeof(d)));
  if (s == MF_OK) s = hip_ok(hipMalloc(&st, sizeof(int)));
  if (s != MF_OK) { hipFree(dd); return s; }
  hipMemcpy(dd, &d, sizeof(d), hipMemcpyHostToDevice);
  hipMemset(st, 0, sizeof(int));
  mfh::launch_gj_inverse(dd, 1, n, st, nullptr);
  s = hip_ok(hipDeviceSynchronize());
  if (s == MF_OK && status_out) hipMemcpy(status_out, st, sizeof(int), hipMemcpyDeviceToHost);
  hipFree(dd);
  hipFree(st);
  return s;
}

mf_status mfh_test_skeleton(int32_t precision, void* F, int32_t ld, int32_t r0, int32_t nr, int32_t c0, int32_t nc,
                            const int32_t* I, int32_t nI, const int32_t* J, int32_t nJ, double eps, int32_t adaptive,
                            int32_t cap, void* U, void* V, int32_t* rank_out) {
  const int maxset = precision == MF_FP64 ? 128 : 192;
  if (nr < 1 || nc < 1 || nI < 0 || nJ < 0 || nI > maxset || nJ > maxset || nI > nr || nJ > nc || cap < 1 ||
      nr + nc > 160 * 1024 || cap < (nI < nJ ? nI : nJ) || !F || !U || !V || !rank_out)
    return MF_EINVAL;
  if (precision == MF_FP64)
    return skel_t<double>(F, ld, r0, nr, c0, nc, I, nI, J, nJ, eps, adaptive, cap, U, V, rank_out);
  return skel_t<float>(F, ld, r0, nr, c0, nc, I, nI, J, nJ, eps, adaptive, cap, U, V, rank_out);
}

}  // extern "C"

extern "C" mf_status mfh_test_record_block_errors(int32_t on) {
  mfh::set_record_block_errors(on != 0);
  return MF_OK;
}

extern "C" mf_status mfh_test_phase2_wait(int64_t ticks) {
  mfh::set_phase2_wait_ticks((long long)ticks);
  return MF_OK;
}
