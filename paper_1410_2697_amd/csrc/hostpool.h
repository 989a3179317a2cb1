// Persistent host worker threads shared by the library's host-side work
// (symbolic analysis loops, BDLR set construction beside the device
// factorization).  Threads are created once per process: creating and
// joining a thread per parallel loop costs far more than the loops here.
#pragma once
#include <atomic>
#include <condition_variable>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <type_traits>
#include <vector>

namespace mfh {

// Counts submitted tasks; wait() runs queued pool tasks while it waits, so a
// waiter never blocks the tasks it waits for.
class TaskGroup {
 public:
  void add(int k = 1);
  void done();
  void wait();

 private:
  std::mutex mu_;
  std::condition_variable cv_;
  int left_ = 0;
};

class HostPool {
 public:
  static HostPool& get();
  // number of threads that can run tasks at once, the caller included
  int width() const { return (int)th_.size() + 1; }
  void submit(std::function<void()> f);
  // runs one queued task on the calling thread; false when the queue is empty
  bool run_one();
  ~HostPool();

 private:
  explicit HostPool(int workers);
  void loop();
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::function<void()>> q_;
  std::vector<std::thread> th_;
  bool stop_ = false;
};

// Runs f(begin, end, chunk) over [0, n) in up to width() contiguous chunks
// (one when n < 2 min_chunk); chunk indices are distinct, so per-chunk
// scratch indexed by them is never shared.  The caller takes chunks too, so
// every chunk has been claimed when its own loop ends; it then waits only for
// chunks other threads are running, never runs unrelated queued tasks (which
// may be long), and helper tasks that start late find no chunk left.
template <typename F>
void parallel_for(int n, int min_chunk, F&& f) {
  HostPool& pool = HostPool::get();
  const int nt = std::max(1, std::min(pool.width(), n / std::max(1, min_chunk)));
  if (nt <= 1) {
    if (n > 0) f(0, n, 0);
    return;
  }
  struct State {
    std::atomic<int> next{0}, done{0};
  };
  auto state = std::make_shared<State>();
  const int ch = (n + nt - 1) / nt;
  // claims and runs chunks; f is only touched while a chunk is unfinished,
  // which keeps the caller (and f) waiting below
  using Fn = typename std::remove_reference<F>::type;
  Fn* fp = &f;
  auto run = [n, nt, ch, fp](State* s) {
    for (;;) {
      const int c = s->next.fetch_add(1);
      if (c >= nt) return;
      const int b = c * ch, e = std::min(n, b + ch);
      if (b < e) (*fp)(b, e, c);
      s->done.fetch_add(1, std::memory_order_release);
    }
  };
  for (int t = 1; t < nt; ++t) pool.submit([state, run]() { run(state.get()); });
  run(state.get());
  while (state->done.load(std::memory_order_acquire) < nt) std::this_thread::yield();
}

// threads the host-side loops use at most
inline int max_workers() { return HostPool::get().width(); }

}  // namespace mfh
