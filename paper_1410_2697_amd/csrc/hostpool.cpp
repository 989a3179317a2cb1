#include "hostpool.h"

#include <algorithm>
#include <chrono>

namespace mfh {

void TaskGroup::add(int k) {
  std::lock_guard<std::mutex> g(mu_);
  left_ += k;
}

void TaskGroup::done() {
  std::lock_guard<std::mutex> g(mu_);
  if (--left_ == 0) cv_.notify_all();
}

void TaskGroup::wait() {
  HostPool& pool = HostPool::get();
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu_);
      if (left_ == 0) return;
    }
    if (pool.run_one()) continue;
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait_for(lk, std::chrono::microseconds(200), [&] { return left_ == 0; });
    if (left_ == 0) return;
  }
}

HostPool& HostPool::get() {
  // at least one worker: the factorization's level loop waits for BDLR
  // tasks without running them itself
  static HostPool pool(std::max(1, std::min<int>((int)std::thread::hardware_concurrency(), 16) - 1));
  return pool;
}

HostPool::HostPool(int workers) {
  for (int i = 0; i < workers; ++i) th_.emplace_back([this]() { loop(); });
}

HostPool::~HostPool() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  for (auto& t : th_) t.join();
}

void HostPool::submit(std::function<void()> f) {
  {
    std::lock_guard<std::mutex> g(mu_);
    q_.push_back(std::move(f));
  }
  cv_.notify_one();
}

bool HostPool::run_one() {
  std::function<void()> f;
  {
    std::lock_guard<std::mutex> g(mu_);
    if (q_.empty()) return false;
    f = std::move(q_.front());
    q_.pop_front();
  }
  f();
  return true;
}

void HostPool::loop() {
  for (;;) {
    std::function<void()> f;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return stop_ || !q_.empty(); });
      if (stop_ && q_.empty()) return;
      f = std::move(q_.front());
      q_.pop_front();
    }
    f();
  }
}

}  // namespace mfh
