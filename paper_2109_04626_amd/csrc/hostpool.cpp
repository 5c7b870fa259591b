// A small persistent pool of host threads for the library's host-side
// loops (candidate sets, deletion decoding, per-instance work in a batch):
// the workers are started once and reused, so a skeleton call does not pay
// thread creation at every level.  One job runs at a time; a call made
// while the pool is busy, or from inside a job, runs inline.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "fpc_internal.h"

namespace fpc {

namespace {

class HostPool {
  public:
    HostPool()
    {
        const unsigned hw = std::thread::hardware_concurrency();
        const int n = (int)std::min<unsigned>(hw ? hw : 1, 16u) - 1;  // the caller is one more worker
        for (int t = 0; t < n; ++t) workers_.emplace_back([this] { loop(); });
    }
    ~HostPool()
    {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &w : workers_) w.join();
    }
    int size() const { return (int)workers_.size() + 1; }

    // fn(k) for k in [0, n); returns when every k is done.
    void run(int n, const std::function<void(int)> &fn)
    {
        std::unique_lock<std::mutex> busy(job_m_, std::try_to_lock);
        if (!busy.owns_lock() || in_job_ || workers_.empty() || n <= 1) {
            for (int k = 0; k < n; ++k) fn(k);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(m_);
            fn_ = &fn;
            n_ = n;
            next_.store(0);
            pending_ = (int)workers_.size();
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> lk(m_);
        done_cv_.wait(lk, [this] { return pending_ == 0; });
        fn_ = nullptr;
    }

  private:
    void work()
    {
        in_job_ = true;
        for (int k = next_++; k < n_; k = next_++) (*fn_)(k);
        in_job_ = false;
    }
    void loop()
    {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
            }
            work();
            {
                std::lock_guard<std::mutex> lk(m_);
                if (--pending_ == 0) done_cv_.notify_one();
            }
        }
    }

    std::vector<std::thread> workers_;
    std::mutex m_, job_m_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int)> *fn_ = nullptr;
    int n_ = 0;
    std::atomic<int> next_{0};
    int pending_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
    static thread_local bool in_job_;
};

thread_local bool HostPool::in_job_ = false;

HostPool &pool()
{
    static HostPool p;
    return p;
}

}  // namespace

void host_parallel(int n, const std::function<void(int)> &fn) { pool().run(n, fn); }

int host_threads() { return pool().size(); }

}  // namespace fpc
