// Request server (include/mfh.h, "Serving"): requests are analysed on the
// submitting thread, queued with their estimated peak device bytes, and
// admitted in arrival order by worker threads, one HIP stream each, as soon
// as the head request fits the memory budget beside the running requests and
// the resident factors.  Admitted requests factor and solve concurrently on
// their streams.
#include "server.h"

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <iterator>

namespace mfh {
namespace {
double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

Server::Server(const mf_server_opts& o) : o_(o) {
  if (o_.slots < 1 || o_.slots > 16) throw Err{MF_EINVAL, "slots must be 1..16"};
  if (!(o_.tol > 0.0)) throw Err{MF_EINVAL, "tol must be > 0"};
  if (hipGetDevice(&dev_) != hipSuccess) {
    (void)hipGetLastError();
    throw Err{MF_ESTATE, "no HIP device is visible"};
  }
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    throw Err{MF_EHIP, "hipMemGetInfo failed"};
  }
  device_total_ = (int64_t)tot;
  budget_ = o_.mem_budget;
  if (budget_ <= 0) budget_ = (int64_t)(0.8 * (double)fr);
  for (int i = 0; i < o_.slots; ++i) workers_.emplace_back([this]() { worker(); });
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
    for (int64_t id : queue_) {
      Req& r = *reqs_[id];
      r.state = 2;
      r.status = MF_ESTATE;
      r.err = "server stopped before the request ran";
    }
    queue_.clear();
  }
  cv_work_.notify_all();
  cv_done_.notify_all();
  for (auto& t : workers_) t.join();
  factors_.clear();   // each factor waits for its own streams' work before freeing
}

int64_t Server::solve_bytes(int n, int nrhs) const {
  const int m = std::max(1, o_.gmres.restart);
  return (int64_t)(8.0 * n * nrhs * (2.0 * m + 6.0)) + (16 << 20);
}

int64_t Server::submit(int n, const int32_t* rowptr, const int32_t* colind, const double* vals,
                       const double* coords, int dim, int nrhs, const double* b) {
  if (n < 1 || !rowptr || !colind || !vals || !coords || !b || nrhs < 1) throw Err{MF_EINVAL, "bad request"};
  auto r = std::make_unique<Req>();
  r->t_submit = now();
  r->sym = std::make_unique<Symbolic>();
  const std::string e = analyze(n, rowptr, colind, coords, dim, o_.leaf, *r->sym);
  if (!e.empty()) throw Err{MF_EINVAL, e};
  r->info.t_analyze = now() - r->t_submit;
  r->n = n;
  r->nrhs = nrhs;
  r->vals.assign(vals, vals + r->sym->nnz);
  r->b.assign(b, b + (size_t)n * nrhs);
  int64_t pers = 0, peak = 0;
  estimate_bytes(*r->sym, o_.factor, nrhs, o_.gmres.restart, pers, peak);
  r->est = std::max(peak, pers);
  r->info.est_bytes = r->est;
  // a request larger than the whole device can never run, not even alone
  if (r->est > device_total_)
    throw Err{MF_EBUDGET, "estimated device bytes " + std::to_string(r->est) + " exceed the device's " +
                              std::to_string(device_total_)};
  std::lock_guard<std::mutex> g(mu_);
  if (stop_) throw Err{MF_ESTATE, "server stopped"};
  r->id = next_id_++;
  const int64_t id = r->id;
  queue_.push_back(id);
  reqs_[id] = std::move(r);
  cv_work_.notify_all();
  return id;
}

int64_t Server::resolve(int64_t factor_ticket, int nrhs, const double* b) {
  if (!b || nrhs < 1) throw Err{MF_EINVAL, "bad request"};
  std::lock_guard<std::mutex> g(mu_);
  if (stop_) throw Err{MF_ESTATE, "server stopped"};
  auto it = factors_.find(factor_ticket);
  if (it == factors_.end() || it->second->released) throw Err{MF_ESTATE, "no resident factor for this ticket"};
  Factor& f = *it->second;
  auto r = std::make_unique<Req>();
  r->t_submit = now();
  r->resolve = true;
  r->factor_id = factor_ticket;
  r->n = f.n;
  r->nrhs = nrhs;
  r->b.assign(b, b + (size_t)f.n * nrhs);
  r->est = solve_bytes(f.n, nrhs);
  r->info.est_bytes = r->est;
  ++f.users;                      // pinned until the solve is done
  r->id = next_id_++;
  const int64_t id = r->id;
  queue_.push_back(id);
  reqs_[id] = std::move(r);
  cv_work_.notify_all();
  return id;
}

// A factor handle serves one solve at a time (its GMRES workspaces and apply
// plans are shared by every solve on it), so a resolve waits while another
// resolve of the same factor runs; requests behind it may go first.  Memory
// admission keeps arrival order: the first request that does not fit stops
// the scan.
std::deque<int64_t>::iterator Server::pick_locked(std::vector<std::unique_ptr<Factor>>& evicted) {
  for (auto it = queue_.begin(); it != queue_.end(); ++it) {
    Req& r = *reqs_[*it];
    if (r.resolve) {
      auto f = factors_.find(r.factor_id);
      if (f != factors_.end() && f->second->busy) continue;
    }
    return admit_locked(r, evicted) ? it : queue_.end();
  }
  return queue_.end();
}

bool Server::admit_locked(Req& r, std::vector<std::unique_ptr<Factor>>& evicted) {
  for (;;) {
    if (in_use_ + r.est <= budget_) return true;
    // drop the least recently used resident factor nobody is using
    auto lru = factors_.end();
    for (auto it = factors_.begin(); it != factors_.end(); ++it)
      if (it->second->users == 0 && (lru == factors_.end() || it->second->last_use < lru->second->last_use))
        lru = it;
    if (lru == factors_.end()) break;
    in_use_ -= lru->second->bytes;
    evicted.push_back(std::move(lru->second));
    factors_.erase(lru);
  }
  return running_ == 0;           // larger than the whole budget: run alone
}

// Requests that join an admitted submit request: the ones queued right
// behind it, in arrival order, while each is a submit request, the group
// stays within `merge` requests and kMergeCols right-hand sides, and the
// summed estimates plus the merged solve's vectors fit the budget; the
// first that does not qualify ends the group.
int64_t Server::group_locked(std::deque<int64_t>::iterator it, std::vector<int64_t>& ids) {
  constexpr int kMergeCols = 16;
  const Req& h = *reqs_[*it];
  ids.assign(1, *it);
  int64_t est = h.est;
  if (h.resolve || o_.keep_factors || o_.merge <= 1 || h.nrhs > kMergeCols) return est;
  int64_t n = h.n;
  int cols = h.nrhs;
  for (auto q = std::next(it); q != queue_.end() && (int)ids.size() < o_.merge; ++q) {
    const Req& r = *reqs_[*q];
    if (r.resolve || cols + r.nrhs > kMergeCols || r.sym->leaf != h.sym->leaf || r.sym->dim != h.sym->dim) break;
    const int64_t add = est + r.est + solve_bytes((int)std::min<int64_t>(n + r.n, INT32_MAX), cols + r.nrhs);
    if (in_use_ + add > budget_) break;
    ids.push_back(*q);
    est += r.est;
    n += r.n;
    cols += r.nrhs;
  }
  return ids.size() > 1 ? est + solve_bytes((int)std::min<int64_t>(n, INT32_MAX), cols) : est;
}

void Server::worker() {
  (void)hipSetDevice(dev_);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    st = nullptr;
  }
  DevBuf db, dx;
  for (;;) {
    std::vector<std::unique_ptr<Factor>> evicted;
    std::vector<Req*> group;
    int64_t charge = 0;
    {
      std::unique_lock<std::mutex> lk(mu_);
      auto pick = queue_.end();
      for (;;) {
        if (stop_) break;
        pick = pick_locked(evicted);
        if (pick != queue_.end()) break;
        cv_work_.wait(lk);
      }
      if (stop_) break;
      std::vector<int64_t> ids;
      charge = group_locked(pick, ids);
      for (int64_t id : ids) {
        Req* r = reqs_[id].get();
        queue_.erase(std::find(queue_.begin(), queue_.end(), id));
        if (r->resolve) factors_.at(r->factor_id)->busy = true;
        r->state = 1;
        r->info.t_queue = now() - r->t_submit;
        r->info.group_size = (int32_t)ids.size();
        group.push_back(r);
      }
      in_use_ += charge;
      ++running_;
    }
    evicted.clear();              // waits for their streams, outside the lock
    if (group.size() == 1) run(*group[0], st, db, dx);
    else run_merged(group, st, db, dx);
    {
      std::lock_guard<std::mutex> g(mu_);
      in_use_ -= charge;
      --running_;
      for (Req* r : group) {
        r->state = 2;
        r->info.t_total = now() - r->t_submit;
      }
    }
    cv_done_.notify_all();
    cv_work_.notify_all();
  }
  if (st) {
    (void)hipStreamSynchronize(st);
    db.release();
    dx.release();
    (void)hipStreamDestroy(st);
  }
}

void Server::run(Req& r, hipStream_t st, DevBuf& db, DevBuf& dx) {
  std::unique_ptr<Factor> own;
  Factor* f = nullptr;
  try {
    if (!r.resolve) {
      mf_opts fo = o_.factor;
      fo.stream = st;
      const double t0 = now();
      own = std::make_unique<Factor>();
      own->n = r.n;
      own->sym = std::move(r.sym);
      // A multi-workgroup phase-2 launch needs its workgroups resident at
      // once; should another slot's kernels hold the compute units past the
      // barrier wait, the factorisation gives up cleanly and runs once more.
      for (int attempt = 0;; ++attempt) {
        try {
          own->num = make_numeric(*own->sym, r.vals.data(), fo);
          break;
        } catch (const Err& e) {
          if (attempt > 0 || e.code != MF_EHIP || e.msg.rfind(kPhase2WaitMsg, 0) != 0) throw;
        }
      }
      r.info.t_factor = now() - t0;
      r.info.peak_bytes = own->num->ms.peak;
      r.vals.clear();
      r.vals.shrink_to_fit();
      f = own.get();
    } else {
      std::lock_guard<std::mutex> g(mu_);
      f = factors_.at(r.factor_id).get();
    }
    const double t1 = now();
    const size_t bytes = (size_t)r.n * r.nrhs * sizeof(double);
    db.ensure(bytes, nullptr, st);
    dx.ensure(bytes, nullptr, st);
    HIPCHK(hipMemcpyAsync(db.p, r.b.data(), bytes, hipMemcpyHostToDevice, st));
    mf_gmres_opts go = o_.gmres;
    go.stream = st;
    std::vector<mf_gmres_info> gi(r.nrhs);
    mf_status s = MF_OK;
    f->num->gmres(r.nrhs, db.as<double>(), dx.as<double>(), o_.tol, go, gi.data(), &s);
    r.x.resize((size_t)r.n * r.nrhs);
    HIPCHK(hipMemcpyAsync(r.x.data(), dx.p, bytes, hipMemcpyDeviceToHost, st));
    f->num->note_stream(st);
    HIPCHK(hipStreamSynchronize(st));
    r.info.t_solve = now() - t1;
    for (const auto& i : gi) {
      r.info.iters_max = std::max(r.info.iters_max, i.iters);
      r.info.relres_max = std::max(r.info.relres_max, i.relres);
    }
    r.status = s;
    if (s == MF_ENOCONV) r.err = "GMRES did not reach tol within maxit";
    r.info.resident_bytes = f->num->ms.current;
  } catch (const Err& e) {
    r.status = e.code;
    r.err = e.msg;
  } catch (const std::bad_alloc&) {
    r.status = MF_ENOMEM;
    r.err = "host allocation failed";
  } catch (const std::exception& e) {
    r.status = MF_EINVAL;
    r.err = e.what();
  }
  r.info.status = r.status;
  std::unique_ptr<Factor> drop;
  {
    std::lock_guard<std::mutex> g(mu_);
    if (r.resolve) {
      auto it = factors_.find(r.factor_id);
      if (it != factors_.end()) {
        Factor& rf = *it->second;
        --rf.users;
        rf.busy = false;
        rf.last_use = ++clock_;
        in_use_ += f ? (f->num->ms.current - rf.bytes) : 0;   // a new nrhs may add workspaces
        rf.bytes = f ? f->num->ms.current : rf.bytes;
        if (rf.released && rf.users == 0) {
          in_use_ -= rf.bytes;
          drop = std::move(it->second);
          factors_.erase(it);
        }
      }
    } else if (own && o_.keep_factors && (r.status == MF_OK || r.status == MF_ENOCONV)) {
      own->bytes = own->num->ms.current;
      own->last_use = ++clock_;
      in_use_ += own->bytes;
      factors_[r.id] = std::move(own);
    }
  }
  drop.reset();
  own.reset();
}

void Server::run_merged(const std::vector<Req*>& rs, hipStream_t st, DevBuf& db, DevBuf& dx) {
  const int k = (int)rs.size();
  std::vector<int64_t> no(k + 1, 0);
  std::vector<int> co(k + 1, 0);
  for (int i = 0; i < k; ++i) {
    no[i + 1] = no[i] + rs[i]->n;
    co[i + 1] = co[i] + rs[i]->nrhs;
  }
  const int64_t N = no[k];
  const int C = co[k];
  Symbolic msym;                  // outlives the factor below, which refers to it
  std::unique_ptr<NumericBase> num;
  bool alone = false;             // the merged factorisation failed: each request runs by itself
  try {
    const double t0 = now();
    std::vector<const Symbolic*> parts;
    size_t nv = 0;
    for (Req* r : rs) {
      parts.push_back(r->sym.get());
      nv += r->vals.size();
    }
    const std::string e = merge(parts, msym);
    if (!e.empty()) throw Err{MF_EINVAL, e};
    std::vector<double> vals;
    vals.reserve(nv);
    for (Req* r : rs) vals.insert(vals.end(), r->vals.begin(), r->vals.end());
    mf_opts fo = o_.factor;
    fo.stream = st;
    for (int attempt = 0;; ++attempt) {   // the same single retry as a request alone
      try {
        num = make_numeric(msym, vals.data(), fo);
        break;
      } catch (const Err& e2) {
        if (attempt == 0 && e2.code == MF_EHIP && e2.msg.rfind(kPhase2WaitMsg, 0) == 0) continue;
        // one request of the group may be at fault (a matrix that is not
        // positive definite, say): the others must not share its error
        if (e2.code == MF_ENOTSPD || e2.code == MF_ECAPACITY || e2.code == MF_EINVAL) {
          alone = true;
          break;
        }
        throw;
      }
    }
    if (!alone) {
      const double t_factor = now() - t0;
      // request i's right-hand sides in columns co[i].., zero outside its rows
      const double t1 = now();
      std::vector<double> B((size_t)N * C, 0.0);
      for (int i = 0; i < k; ++i)
        for (int c = 0; c < rs[i]->nrhs; ++c)
          std::copy(rs[i]->b.begin() + (size_t)c * rs[i]->n, rs[i]->b.begin() + (size_t)(c + 1) * rs[i]->n,
                    B.begin() + (size_t)(co[i] + c) * N + no[i]);
      const size_t bytes = (size_t)N * C * sizeof(double);
      db.ensure(bytes, nullptr, st);
      dx.ensure(bytes, nullptr, st);
      HIPCHK(hipMemcpyAsync(db.p, B.data(), bytes, hipMemcpyHostToDevice, st));
      mf_gmres_opts go = o_.gmres;
      go.stream = st;
      std::vector<mf_gmres_info> gi(C);
      std::vector<int32_t> win(2 * (size_t)C);     // each column touches only its request's rows
      for (int i = 0; i < k; ++i)
        for (int c = co[i]; c < co[i + 1]; ++c) {
          win[2 * c] = (int32_t)no[i];
          win[2 * c + 1] = (int32_t)no[i + 1];
        }
      mf_status s = MF_OK;
      num->gmres(C, db.as<double>(), dx.as<double>(), o_.tol, go, gi.data(), &s, win.data());
      HIPCHK(hipMemcpyAsync(B.data(), dx.p, bytes, hipMemcpyDeviceToHost, st));
      num->note_stream(st);
      HIPCHK(hipStreamSynchronize(st));
      const double t_solve = now() - t1;
      for (int i = 0; i < k; ++i) {
        Req& r = *rs[i];
        r.x.resize((size_t)r.n * r.nrhs);
        bool conv = true;
        for (int c = 0; c < r.nrhs; ++c) {
          std::copy(B.begin() + (size_t)(co[i] + c) * N + no[i], B.begin() + (size_t)(co[i] + c) * N + no[i + 1],
                    r.x.begin() + (size_t)c * r.n);
          const mf_gmres_info& g = gi[co[i] + c];
          r.info.iters_max = std::max(r.info.iters_max, g.iters);
          r.info.relres_max = std::max(r.info.relres_max, g.relres);
          conv &= g.converged != 0;
        }
        r.status = conv ? MF_OK : MF_ENOCONV;
        if (!conv) r.err = "GMRES did not reach tol within maxit";
        r.info.t_factor = t_factor;
        r.info.t_solve = t_solve;
        r.info.peak_bytes = num->ms.peak;
      }
    }
  } catch (const Err& e) {
    for (Req* r : rs) { r->status = e.code; r->err = e.msg; }
  } catch (const std::bad_alloc&) {
    for (Req* r : rs) { r->status = MF_ENOMEM; r->err = "host allocation failed"; }
  } catch (const std::exception& e) {
    for (Req* r : rs) { r->status = MF_EINVAL; r->err = e.what(); }
  }
  num.reset();
  if (alone) {                    // factor and solve each request by itself
    for (Req* r : rs) {
      r->info.group_size = 1;
      run(*r, st, db, dx);
    }
    return;
  }
  for (Req* r : rs) {
    r->info.status = r->status;
    r->vals.clear();
    r->vals.shrink_to_fit();
    r->sym.reset();
  }
}

void Server::wait(int64_t ticket, double* x, mf_request_info* info) {
  std::unique_ptr<Req> r;
  {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) throw Err{MF_EINVAL, "unknown ticket (or already waited for)"};
    Req* p = it->second.get();
    cv_done_.wait(lk, [&] { return p->state == 2; });
    r = std::move(it->second);
    reqs_.erase(it);
  }
  if (info) *info = r->info;
  if (x && !r->x.empty()) std::copy(r->x.begin(), r->x.end(), x);
  if (r->status != MF_OK) throw Err{r->status, r->err};
}

void Server::release(int64_t factor_ticket) {
  std::unique_ptr<Factor> drop;
  {
    std::lock_guard<std::mutex> g(mu_);
    auto it = factors_.find(factor_ticket);
    if (it == factors_.end()) throw Err{MF_EINVAL, "no resident factor for this ticket"};
    it->second->released = true;
    if (it->second->users == 0) {
      in_use_ -= it->second->bytes;
      drop = std::move(it->second);
      factors_.erase(it);
    }
  }
  cv_work_.notify_all();
}

void Server::memory(int64_t* in_use, int64_t* budget) {
  std::lock_guard<std::mutex> g(mu_);
  if (in_use) *in_use = in_use_;
  if (budget) *budget = budget_;
}

}  // namespace mfh
