// A small persistent pool of host threads for the library's host-side
// loops (candidate sets, deletion decoding, per-instance work in a batch):
// the workers are started once and reused, so a skeleton call does not pay
// thread creation at every level.  One job runs at a time; a call made
// while the pool is busy, or from inside a job, runs inline.
//
// Between jobs a worker spins on the job counter for a short while before
// it sleeps, so the back-to-back jobs of one level start without a wake-up;
// the caller takes items too and returns once every item is done and no
// worker still holds the job, without waiting for sleeping workers.  A
// caller about to need the pool after a device wait wakes the sleepers
// beforehand (wake), so that they spin when the job comes.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "fpc_internal.h"

namespace fpc {

namespace {

inline void cpu_relax() { __builtin_ia32_pause(); }

class HostPool {
  public:
    HostPool()
    {
        // the caller is one more worker, and one core is left to the runtime's
        // own threads and the result prefetch (spinning workers must not
        // take every core of the process's share)
        const unsigned hw = std::thread::hardware_concurrency();
        const int n = std::max(0, (int)std::min<unsigned>(hw ? hw : 1, 16u) - 2);
        for (int t = 0; t < n; ++t) workers_.emplace_back([this] { loop(); });
    }
    ~HostPool()
    {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_.store(true);
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
        const uint64_t g = gen_.load(std::memory_order_relaxed) + 1;
        Job &J = jobs_[g & 1];
        // a worker that read an older count may still be registered on
        // this slot for a moment (it leaves without touching the job)
        while (J.active.load(std::memory_order_acquire) != 0) cpu_relax();
        J.fn = &fn;
        J.n = n;
        J.next.store(0, std::memory_order_relaxed);
        J.done.store(0, std::memory_order_relaxed);
        {
            std::lock_guard<std::mutex> lk(m_);
            gen_.store(g, std::memory_order_release);
        }
        if (sleepers_.load(std::memory_order_acquire) > 0) cv_.notify_all();
        in_job_ = true;
        work(J);
        in_job_ = false;
        while (J.done.load(std::memory_order_acquire) < n || J.active.load(std::memory_order_acquire) != 0)
            cpu_relax();
    }

    // Sleeping workers start another spin (no job).
    void wake()
    {
        if (sleepers_.load(std::memory_order_acquire) == 0) return;
        {
            std::lock_guard<std::mutex> lk(m_);
            wake_.fetch_add(1, std::memory_order_relaxed);
        }
        cv_.notify_all();
    }

  private:
    struct Job {
        const std::function<void(int)> *fn = nullptr;
        int n = 0;
        std::atomic<int> next{0}, done{0}, active{0};
    };

    static void work(Job &J)
    {
        for (int k = J.next.fetch_add(1, std::memory_order_relaxed); k < J.n;
             k = J.next.fetch_add(1, std::memory_order_relaxed)) {
            (*J.fn)(k);
            J.done.fetch_add(1, std::memory_order_release);
        }
    }

    void loop()
    {
        using clk = std::chrono::steady_clock;
        uint64_t seen = 0;
        for (;;) {
            uint64_t g = gen_.load(std::memory_order_acquire);
            if (g == seen) {
                const auto t0 = clk::now();
                int spins = 0;
                while ((g = gen_.load(std::memory_order_acquire)) == seen && !stop_.load(std::memory_order_relaxed)) {
                    cpu_relax();
                    if ((++spins & 255) == 0 && clk::now() - t0 > std::chrono::microseconds(kSpinUs)) {
                        std::unique_lock<std::mutex> lk(m_);
                        sleepers_.fetch_add(1, std::memory_order_acq_rel);
                        const uint64_t w0 = wake_.load(std::memory_order_relaxed);
                        cv_.wait(lk, [&] {
                            return stop_.load() || gen_.load() != seen || wake_.load(std::memory_order_relaxed) != w0;
                        });
                        sleepers_.fetch_sub(1, std::memory_order_acq_rel);
                        break;
                    }
                }
                if (stop_.load()) return;
                continue;  // read the count again
            }
            Job &J = jobs_[g & 1];
            J.active.fetch_add(1, std::memory_order_acq_rel);
            if (gen_.load(std::memory_order_acquire) != g) {  // a newer job was published meanwhile
                J.active.fetch_sub(1, std::memory_order_release);
                continue;
            }
            seen = g;
            in_job_ = true;
            work(J);
            in_job_ = false;
            J.active.fetch_sub(1, std::memory_order_release);
        }
    }

    static constexpr int kSpinUs = 1000;  // spin this long after a job (or a wake) before sleeping
    std::vector<std::thread> workers_;
    std::mutex m_, job_m_;
    std::condition_variable cv_;
    Job jobs_[2];
    std::atomic<uint64_t> gen_{0}, wake_{0};
    std::atomic<int> sleepers_{0};
    std::atomic<bool> stop_{false};
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

void host_wake() { pool().wake(); }

}  // namespace fpc
