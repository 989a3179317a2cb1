// Request server: continuous batching of independent factor + solve jobs
// (include/mfh.h, "Serving").
#pragma once
#include <hip/hip_runtime.h>

#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mfh.h"
#include "numeric.h"
#include "symbolic.h"

namespace mfh {

class Server {
 public:
  explicit Server(const mf_server_opts& o);
  ~Server();
  int64_t submit(int n, const int32_t* rowptr, const int32_t* colind, const double* vals, const double* coords,
                 int dim, int nrhs, const double* b);
  int64_t resolve(int64_t factor_ticket, int nrhs, const double* b);
  // blocks until done; copies x; throws Err carrying the request's status
  void wait(int64_t ticket, double* x, mf_request_info* info);
  void release(int64_t factor_ticket);
  void memory(int64_t* in_use, int64_t* budget);

 private:
  struct Factor {
    std::unique_ptr<Symbolic> sym;
    std::unique_ptr<NumericBase> num;
    int n = 0;
    int64_t bytes = 0;      // accounted while resident
    int users = 0;          // queued or running resolves
    bool busy = false;      // a resolve is running on it (one solve per factor at a time)
    uint64_t last_use = 0;
    bool released = false;
  };
  struct Req {
    int64_t id = 0;
    bool resolve = false;
    int64_t factor_id = 0;
    int n = 0, nrhs = 0;
    std::unique_ptr<Symbolic> sym;
    std::vector<double> vals, b, x;
    int64_t est = 0;
    int state = 0;          // 0 queued, 1 running, 2 done
    mf_status status = MF_OK;
    std::string err;
    mf_request_info info{};
    double t_submit = 0;
  };

  void worker();
  void run(Req& r, hipStream_t st, DevBuf& db, DevBuf& dx);
  // several submitted requests factored and solved as one block-diagonal system
  void run_merged(const std::vector<Req*>& rs, hipStream_t st, DevBuf& db, DevBuf& dx);
  // requests queued right behind the admitted head `it` that join its group
  // (lock held); returns the group's device-byte charge
  int64_t group_locked(std::deque<int64_t>::iterator it, std::vector<int64_t>& ids);
  // next admissible queued request (lock held), or queue_.end(): requests
  // are taken in arrival order, except that a resolve whose factor is busy
  // with another solve is passed over; evicted factors are moved out
  std::deque<int64_t>::iterator pick_locked(std::vector<std::unique_ptr<Factor>>& evicted);
  bool admit_locked(Req& r, std::vector<std::unique_ptr<Factor>>& evicted);
  int64_t solve_bytes(int n, int nrhs) const;

  mf_server_opts o_{};
  int dev_ = 0;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<int64_t> queue_;
  std::map<int64_t, std::unique_ptr<Req>> reqs_;
  std::map<int64_t, std::unique_ptr<Factor>> factors_;
  int64_t next_id_ = 1, in_use_ = 0, budget_ = 0, device_total_ = 0;
  uint64_t clock_ = 0;
  int running_ = 0;
  bool stop_ = false;
  std::vector<std::thread> workers_;
};

}  // namespace mfh
