// C ABI entry points (include/mfh.h).  Converts exceptions into status codes
// and keeps a per-thread message for mf_last_error().
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <string>

#include "../../include/mfh.h"
#include "../../include/mfh_testing.h"
#include "numeric.h"
#include "prof.h"
#include "server.h"
#include "symbolic.h"

struct mf_symbolic_s {
  mfh::Symbolic s;
};
struct mf_server_s {
  std::unique_ptr<mfh::Server> s;
};
struct mf_numeric_s {
  std::unique_ptr<mfh::NumericBase> n;
};

namespace {
thread_local std::string g_err;
mf_status fail(mf_status c, const std::string& m) {
  g_err = m;
  return c;
}
mf_status gpu_present() {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n < 1) {
    (void)hipGetLastError();
    return fail(MF_ESTATE, "no HIP device is visible");
  }
  return MF_OK;
}
template <typename V>
mf_status export_vec(const V& v, int32_t* buf, int64_t cap, int64_t* len) {
  if (len) *len = (int64_t)v.size();
  if (!buf) return MF_OK;
  if (cap < (int64_t)v.size()) return fail(MF_EINVAL, "export buffer too small");
  for (size_t i = 0; i < v.size(); ++i) buf[i] = (int32_t)v[i];
  return MF_OK;
}
}  // namespace

#define MF_GUARD_BEGIN try {
#define MF_GUARD_END                                                   \
  }                                                                    \
  catch (const mfh::Err& e) { return fail(e.code, e.msg); }            \
  catch (const std::bad_alloc&) { return fail(MF_ENOMEM, "host allocation failed"); } \
  catch (const std::exception& e) { return fail(MF_EINVAL, e.what()); }

extern "C" {

mf_status mf_opts_default(mf_opts* o) {
  if (!o) return fail(MF_EINVAL, "null opts");
  std::memset(o, 0, sizeof(*o));
  o->method = MF_METHOD_HODLR;
  o->precision = MF_FP32;
  o->n_c = 0;
  o->bdlr_depth = -1;
  o->bdlr_cap = 0;
  o->adaptive = 1;
  o->rank_cap = 512;
  o->apply_graph = 4;
  o->eps = 1e-4;
  o->stream = nullptr;
  return MF_OK;
}

mf_status mf_gmres_opts_default(mf_gmres_opts* o) {
  if (!o) return fail(MF_EINVAL, "null opts");
  o->restart = 30;
  o->maxit = 4000;
  o->stream = nullptr;
  return MF_OK;
}

mf_status mf_analyze(int32_t n, const int32_t* rowptr, const int32_t* colind, const double* coords, int32_t dim,
                     int32_t leaf, mf_symbolic_t** out) {
  MF_GUARD_BEGIN
  if (!out) return fail(MF_EINVAL, "null output handle");
  *out = nullptr;
  if (n < 1 || !rowptr || !colind || !coords) return fail(MF_EINVAL, "null or empty input");
  auto h = std::make_unique<mf_symbolic_s>();
  std::string e = mfh::analyze(n, rowptr, colind, coords, dim, leaf, h->s);
  if (!e.empty()) return fail(MF_EINVAL, e);
  *out = h.release();
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_symbolic_merge(const mf_symbolic_t* const* parts, int32_t count, mf_symbolic_t** out) {
  MF_GUARD_BEGIN
  if (!out) return fail(MF_EINVAL, "null output handle");
  *out = nullptr;
  if (!parts || count < 1) return fail(MF_EINVAL, "no analyses to merge");
  std::vector<const mfh::Symbolic*> v(count);
  for (int i = 0; i < count; ++i) {
    if (!parts[i]) return fail(MF_EINVAL, "null analysis handle");
    v[i] = &parts[i]->s;
  }
  auto h = std::make_unique<mf_symbolic_s>();
  std::string e = mfh::merge(v, h->s);
  if (!e.empty()) return fail(MF_EINVAL, e);
  *out = h.release();
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_symbolic_get_info(const mf_symbolic_t* sh, mf_symbolic_info* info) {
  if (!sh || !info) return fail(MF_EINVAL, "null argument");
  const mfh::Symbolic& s = sh->s;
  info->n = s.n;
  info->nnz = s.nnz;
  info->nfronts = (int64_t)s.fronts.size();
  info->nlevels = (int64_t)s.levels.size();
  int64_t mf = 0, mp = 0;
  for (auto& f : s.fronts) { mf = std::max<int64_t>(mf, f.n()); mp = std::max<int64_t>(mp, f.npiv); }
  info->max_front = mf;
  info->max_npiv = mp;
  return MF_OK;
}

mf_status mf_symbolic_export(const mf_symbolic_t* sh, int32_t what, int32_t* buf, int64_t cap, int64_t* len) {
  MF_GUARD_BEGIN
  if (!sh) return fail(MF_EINVAL, "null handle");
  const mfh::Symbolic& s = sh->s;
  std::vector<int64_t> v;
  switch (what) {
    case MF_EXP_PERM: return export_vec(s.perm, buf, cap, len);
    case MF_EXP_FRONT:
      for (auto& f : s.fronts) {
        v.push_back(f.start); v.push_back(f.npiv); v.push_back(f.nf());
        v.push_back(f.parent); v.push_back(f.height); v.push_back((int64_t)f.children.size());
      }
      return export_vec(v, buf, cap, len);
    case MF_EXP_UPD:
      for (auto& f : s.fronts) v.insert(v.end(), f.upd.begin(), f.upd.end());
      return export_vec(v, buf, cap, len);
    case MF_EXP_UPD_PTR:
      v.push_back(0);
      for (auto& f : s.fronts) v.push_back(v.back() + f.nf());
      return export_vec(v, buf, cap, len);
    case MF_EXP_RELMAP:
      for (auto& f : s.fronts) {
        if (f.relmap.size() != f.upd.size()) v.insert(v.end(), f.upd.size(), -1);
        else v.insert(v.end(), f.relmap.begin(), f.relmap.end());
      }
      return export_vec(v, buf, cap, len);
    case MF_EXP_ASM: {
      mfh::bigvec<int> af, ar, ac, as;
      mfh::assembly_map(s, af, ar, ac, as);
      for (size_t e = 0; e < as.size(); ++e) {
        v.push_back(af[e]); v.push_back(ar[e]); v.push_back(ac[e]); v.push_back(as[e]);
      }
      return export_vec(v, buf, cap, len);
    }
    case MF_EXP_BLOCKS:
      for (size_t p = 0; p < s.fronts.size(); ++p)
        for (auto& b : s.fronts[p].blocks) {
          v.push_back((int64_t)p); v.push_back(b.kind); v.push_back(b.r0); v.push_back(b.nr);
          v.push_back(b.c0); v.push_back(b.nc); v.push_back(b.level);
        }
      return export_vec(v, buf, cap, len);
    case MF_EXP_BDLR_I:
    case MF_EXP_BDLR_IPTR:
    case MF_EXP_BDLR_J:
    case MF_EXP_BDLR_JPTR:
      if (s.bdlr_depth == -2) return fail(MF_ESTATE, "call mf_symbolic_bdlr first");
      if (what == MF_EXP_BDLR_I) return export_vec(s.bdlr_I, buf, cap, len);
      if (what == MF_EXP_BDLR_IPTR) return export_vec(s.bdlr_Iptr, buf, cap, len);
      if (what == MF_EXP_BDLR_J) return export_vec(s.bdlr_J, buf, cap, len);
      return export_vec(s.bdlr_Jptr, buf, cap, len);
    default: return fail(MF_EINVAL, "unknown export code");
  }
  MF_GUARD_END
}

mf_status mf_symbolic_bdlr(mf_symbolic_t* sh, int32_t depth, int32_t cap) {
  MF_GUARD_BEGIN
  if (!sh) return fail(MF_EINVAL, "null handle");
  if (cap < 1) return fail(MF_EINVAL, "cap must be >= 1");
  mfh::compute_bdlr(sh->s, depth, cap);
  return MF_OK;
  MF_GUARD_END
}

void mf_symbolic_free(mf_symbolic_t* s) { delete s; }

mf_status mf_factor(const mf_symbolic_t* sh, const double* vals, double eps, int32_t leaf, const mf_opts* opts,
                    mf_numeric_t** out) {
  MF_GUARD_BEGIN
  if (!out) return fail(MF_EINVAL, "null output handle");
  *out = nullptr;
  if (!sh || !vals) return fail(MF_EINVAL, "null argument");
  mf_opts o;
  if (opts) o = *opts; else mf_opts_default(&o);
  o.eps = eps;
  if (o.method != MF_METHOD_HODLR && o.method != MF_METHOD_DENSE) return fail(MF_EINVAL, "unknown method");
  if (o.uv_bf16 && o.method != MF_METHOD_HODLR) return fail(MF_EINVAL, "uv_bf16 needs MF_METHOD_HODLR");
  if (o.precision != MF_FP64 && o.precision != MF_FP32) return fail(MF_EINVAL, "unknown precision");
  if (!(eps >= 0.0) || eps >= 1.0) return fail(MF_EINVAL, "eps must be in [0, 1)");
  if (o.apply_graph < 0 || o.apply_graph > (1 << 20)) return fail(MF_EINVAL, "apply_graph must be in [0, 2^20]");
  if (o.apply_split_chunk != 0 && (o.apply_split_chunk < 64 || o.apply_split_chunk > 4096 || o.apply_split_chunk % 64))
    return fail(MF_EINVAL, "apply_split_chunk must be 0 or a multiple of 64 in [64, 4096]");
  if (o.apply_split_target < 0 || o.apply_split_target > 65536)
    return fail(MF_EINVAL, "apply_split_target must be in [0, 65536]");
  if (o.sampled != 0 && o.sampled != 1) return fail(MF_EINVAL, "sampled must be 0 or 1");
  if (o.adaptive < 0 || o.adaptive > 2) return fail(MF_EINVAL, "adaptive must be 0, 1 or 2");
  if (o.sampled && (o.method != MF_METHOD_HODLR || o.adaptive == 1))
    return fail(MF_EINVAL, "the sampled extend-add forms only the BDLR rows and columns: it needs "
                           "MF_METHOD_HODLR and adaptive 0 or 2");
  if (o.adaptive == 2 && !o.sampled) return fail(MF_EINVAL, "adaptive 2 (the sampled cross) needs sampled = 1");
  if (leaf != 0 && leaf != sh->s.leaf) return fail(MF_EINVAL, "leaf must be 0 or the analysis leaf size");
  if (o.method == MF_METHOD_HODLR) {
    if (sh->s.leaf > 128) return fail(MF_EINVAL, "HODLR leaves are limited to 128");
    if (o.bdlr_cap < 0 || o.rank_cap < 1) return fail(MF_EINVAL, "bdlr_cap must be >= 0 and rank_cap >= 1");
    if (o.rank_cap > 512) return fail(MF_EINVAL, "rank_cap is limited to 512");
    const int maxcap = o.precision == MF_FP64 ? 128 : 192;   // B_hat held by one workgroup
    if (o.bdlr_cap == 0) o.bdlr_cap = maxcap;
    if (o.uv_bf16 && o.precision != MF_FP32) return fail(MF_EINVAL, "uv_bf16 needs MF_FP32");
    if (o.bdlr_cap > maxcap) return fail(MF_EINVAL, "bdlr_cap too large for the LDS pivot kernel");
  }
  mf_status g = gpu_present();
  if (g != MF_OK) return g;
  auto h = std::make_unique<mf_numeric_s>();
  h->n = mfh::make_numeric(sh->s, vals, o);
  *out = h.release();
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_factor_get_info(const mf_numeric_t* f, mf_factor_info* info) {
  if (!f || !info) return fail(MF_EINVAL, "null argument");
  *info = f->n->info;
  info->peak_bytes = f->n->ms.peak;
  info->resident_bytes = f->n->ms.current;
  return MF_OK;
}

mf_status mf_factor_ranks(const mf_numeric_t* f, int32_t* buf, int64_t cap, int64_t* len) {
  if (!f) return fail(MF_EINVAL, "null handle");
  return export_vec(f->n->ranks, buf, cap, len);
}

void mf_factor_free(mf_numeric_t* f) { delete f; }

mf_status mf_apply(mf_numeric_t* f, int32_t nrhs, const double* r, double* z, void* stream) {
  MF_GUARD_BEGIN
  if (!f || !r || !z || nrhs < 1) return fail(MF_EINVAL, "bad argument");
  if (r == z) return fail(MF_EINVAL, "r and z may not alias");
  f->n->apply(nrhs, r, z, static_cast<hipStream_t>(stream));
  f->n->note_stream(static_cast<hipStream_t>(stream));
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_apply_noalloc(mf_numeric_t* f, int32_t nrhs, const double* r, double* z, void* stream) {
  MF_GUARD_BEGIN
  if (!f || !r || !z || nrhs < 1) return fail(MF_EINVAL, "bad argument");
  if (r == z) return fail(MF_EINVAL, "r and z may not alias");
  f->n->apply_noalloc(nrhs, r, z, static_cast<hipStream_t>(stream));
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_direct_solve(mf_numeric_t* f, int32_t nrhs, const double* b, double* x, int32_t refine, void* stream,
                          mf_gmres_info* info) {
  MF_GUARD_BEGIN
  if (!f || !b || !x || nrhs < 1 || b == x) return fail(MF_EINVAL, "bad argument");
  if (refine < 0 || refine > 64) return fail(MF_EINVAL, "refine must be 0..64");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  f->n->direct_solve(nrhs, b, x, refine, st, info);
  f->n->note_stream(st);
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_pcg_opts_default(mf_pcg_opts* o) {
  if (!o) return fail(MF_EINVAL, "null opts");
  *o = mf_pcg_opts{};
  o->maxit = 4000;
  return MF_OK;
}

mf_status pcg_solve(mf_numeric_t* f, int32_t nrhs, const double* b, double* x, double tol, const mf_pcg_opts* opts,
                    mf_gmres_info* info) {
  MF_GUARD_BEGIN
  if (!f || !b || !x || nrhs < 1 || b == x) return fail(MF_EINVAL, "bad argument");
  if (!(tol > 0.0)) return fail(MF_EINVAL, "tol must be > 0");
  mf_pcg_opts o;
  if (opts) o = *opts; else mf_pcg_opts_default(&o);
  if (o.maxit < 1 || o.reserved != 0) return fail(MF_EINVAL, "maxit must be >= 1 and reserved 0");
  mf_status s = MF_OK;
  const hipStream_t st = static_cast<hipStream_t>(o.stream);
  f->n->pcg(nrhs, b, x, tol, o.maxit, st, info, &s);
  f->n->note_stream(st);
  if (s == MF_ENOCONV) return fail(MF_ENOCONV, "PCG did not reach tol within maxit");
  return s;
  MF_GUARD_END
}

mf_status mf_spmv(mf_numeric_t* f, int32_t nrhs, const double* x, double* y, void* stream) {
  MF_GUARD_BEGIN
  if (!f || !x || !y || nrhs < 1 || x == y) return fail(MF_EINVAL, "bad argument");
  f->n->spmv(nrhs, x, y, 1.0, 0.0, static_cast<hipStream_t>(stream));
  f->n->note_stream(static_cast<hipStream_t>(stream));
  return MF_OK;
  MF_GUARD_END
}

mf_status gmres_solve(mf_numeric_t* f, int32_t nrhs, const double* b, double* x, double tol,
                      const mf_gmres_opts* opts, mf_gmres_info* info) {
  MF_GUARD_BEGIN
  if (!f || !b || !x || nrhs < 1 || b == x) return fail(MF_EINVAL, "bad argument");
  if (!(tol > 0.0)) return fail(MF_EINVAL, "tol must be > 0");
  mf_gmres_opts o;
  if (opts) o = *opts; else mf_gmres_opts_default(&o);
  if (o.restart < 1 || o.restart > 60 || o.maxit < 1) return fail(MF_EINVAL, "restart must be 1..60, maxit >= 1");
  mf_status s = MF_OK;
  f->n->gmres(nrhs, b, x, tol, o, info, &s);
  f->n->note_stream(static_cast<hipStream_t>(o.stream));
  if (s == MF_ENOCONV) return fail(MF_ENOCONV, "GMRES did not reach tol within maxit");
  return s;
  MF_GUARD_END
}

mf_status mfh_test_block_errors(const mf_numeric_t* f, double* out, int64_t cap, int64_t* count) {
  MF_GUARD_BEGIN
  if (!f || !count || cap < 0 || (cap > 0 && !out)) return fail(MF_EINVAL, "bad argument");
  const auto& e = f->n->block_errors;
  *count = (int64_t)e.size();
  for (int64_t i = 0; i < std::min<int64_t>(cap, (int64_t)e.size()); ++i) {
    double* o = out + 6 * i;
    o[0] = e[i].front; o[1] = e[i].block; o[2] = e[i].rank;
    o[3] = e[i].bmax; o[4] = e[i].u11; o[5] = e[i].emax;
  }
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_estimate_bytes(const mf_symbolic_t* sym, const mf_opts* opts, int32_t nrhs, int32_t restart,
                            int64_t* persistent, int64_t* peak) {
  MF_GUARD_BEGIN
  if (!sym || nrhs < 1 || restart < 1) return fail(MF_EINVAL, "bad argument");
  mf_opts o;
  if (opts) o = *opts; else mf_opts_default(&o);
  if (o.rank_cap < 1) return fail(MF_EINVAL, "rank_cap must be >= 1");
  int64_t pe = 0, pk = 0;
  mfh::estimate_bytes(sym->s, o, nrhs, restart, pe, pk);
  if (persistent) *persistent = pe;
  if (peak) *peak = pk;
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_server_opts_default(mf_server_opts* o) {
  if (!o) return fail(MF_EINVAL, "null opts");
  std::memset(o, 0, sizeof(*o));
  o->slots = 4;
  o->leaf = 128;
  o->mem_budget = 0;
  o->tol = 1e-10;
  mf_opts_default(&o->factor);
  mf_gmres_opts_default(&o->gmres);
  o->keep_factors = 0;
  o->merge = 1;
  return MF_OK;
}

mf_status mf_server_create(const mf_server_opts* o, mf_server_t** out) {
  MF_GUARD_BEGIN
  if (!out) return fail(MF_EINVAL, "null out");
  *out = nullptr;
  mf_server_opts so;
  if (o) so = *o; else mf_server_opts_default(&so);
  mf_opts& fo = so.factor;
  if (so.leaf < 1) return fail(MF_EINVAL, "leaf must be >= 1");
  if (fo.method == MF_METHOD_HODLR) {
    if (so.leaf > 128) return fail(MF_EINVAL, "HODLR leaves are limited to 128");
    const int maxcap = fo.precision == MF_FP64 ? 128 : 192;
    if (fo.bdlr_cap == 0) fo.bdlr_cap = maxcap;
    if (fo.bdlr_cap < 1 || fo.bdlr_cap > maxcap || fo.rank_cap < 1 || fo.rank_cap > 512)
      return fail(MF_EINVAL, "bdlr_cap or rank_cap out of range");
  }
  if (!(fo.eps >= 0.0) || fo.eps >= 1.0) return fail(MF_EINVAL, "eps must be in [0, 1)");
  if (fo.apply_split_chunk != 0 && (fo.apply_split_chunk < 64 || fo.apply_split_chunk > 4096 || fo.apply_split_chunk % 64))
    return fail(MF_EINVAL, "apply_split_chunk must be 0 or a multiple of 64 in [64, 4096]");
  if (fo.apply_split_target < 0 || fo.apply_split_target > 65536)
    return fail(MF_EINVAL, "apply_split_target must be in [0, 65536]");
  if (so.gmres.restart < 1 || so.gmres.restart > 60 || so.gmres.maxit < 1)
    return fail(MF_EINVAL, "restart must be 1..60, maxit >= 1");
  if (so.merge < 1 || so.merge > 16) return fail(MF_EINVAL, "merge must be 1..16");
  mf_status g = gpu_present();
  if (g != MF_OK) return g;
  auto h = std::make_unique<mf_server_s>();
  h->s = std::make_unique<mfh::Server>(so);
  *out = h.release();
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_server_submit(mf_server_t* sv, int32_t n, const int32_t* rowptr, const int32_t* colind,
                           const double* vals, const double* coords, int32_t dim, int32_t nrhs,
                           const double* b, int64_t* ticket) {
  MF_GUARD_BEGIN
  if (!sv || !ticket) return fail(MF_EINVAL, "null argument");
  *ticket = sv->s->submit(n, rowptr, colind, vals, coords, dim, nrhs, b);
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_server_resolve(mf_server_t* sv, int64_t factor_ticket, int32_t nrhs, const double* b,
                            int64_t* ticket) {
  MF_GUARD_BEGIN
  if (!sv || !ticket) return fail(MF_EINVAL, "null argument");
  *ticket = sv->s->resolve(factor_ticket, nrhs, b);
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_server_wait(mf_server_t* sv, int64_t ticket, double* x, mf_request_info* info) {
  MF_GUARD_BEGIN
  if (!sv) return fail(MF_EINVAL, "null server");
  sv->s->wait(ticket, x, info);
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_server_release(mf_server_t* sv, int64_t factor_ticket) {
  MF_GUARD_BEGIN
  if (!sv) return fail(MF_EINVAL, "null server");
  sv->s->release(factor_ticket);
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_server_memory(mf_server_t* sv, int64_t* in_use, int64_t* budget) {
  if (!sv) return fail(MF_EINVAL, "null server");
  sv->s->memory(in_use, budget);
  return MF_OK;
}

void mf_server_destroy(mf_server_t* sv) { delete sv; }

mf_status mf_prof_start(const char* names) {
  MF_GUARD_BEGIN
  mfh::prof_start(names ? std::string(names) : std::string());
  return MF_OK;
  MF_GUARD_END
}

mf_status mf_prof_stop(mf_kstat* out, int32_t cap, int32_t* n) {
  MF_GUARD_BEGIN
  if (cap < 0 || (cap > 0 && !out)) return fail(MF_EINVAL, "bad output array");
  const auto t = mfh::prof_stop();
  const int m = std::min<int>(cap, (int)t.size());
  for (int i = 0; i < m; ++i) {
    std::memset(&out[i], 0, sizeof(mf_kstat));
    std::strncpy(out[i].name, mfh::prof_name(t[i].kind), sizeof(out[i].name) - 1);
    out[i].launches = t[i].launches;
    out[i].seconds = t[i].seconds;
    out[i].flops = t[i].flops;
    out[i].bytes = t[i].bytes;
  }
  if (n) *n = (int32_t)t.size();
  return MF_OK;
  MF_GUARD_END
}

const char* mf_last_error(void) { return g_err.c_str(); }

}  // extern "C"
