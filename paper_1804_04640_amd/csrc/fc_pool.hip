// Host fork-join for the planners: parallel_for(T, f) runs f(0) on the
// calling thread and f(1) .. f(T - 1) on worker threads that persist for
// the life of the process (created on first use), so a call costs a wake-up
// instead of T - 1 thread creations.  One fork-join uses the workers at a
// time; a call that finds them busy (another host thread planning) creates
// threads of its own for that call.
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "fc_internal.h"

namespace fc {
namespace {

struct Pool {
    std::mutex call;  // held for a whole fork-join
    std::mutex m;
    std::condition_variable wake, done;
    std::vector<std::thread> workers;  // ids 1, 2, ...
    const std::function<void(int)> *job = nullptr;
    int njob = 0;
    int pending = 0;
    uint64_t gen = 0;

    void loop(int id) {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(int)> *f;
            int nj;
            {
                std::unique_lock<std::mutex> l(m);
                wake.wait(l, [&] { return gen != seen; });
                seen = gen;
                f = job;
                nj = njob;
            }
            if (id < nj) {
                (*f)(id);
                std::lock_guard<std::mutex> l(m);
                if (--pending == 0) done.notify_one();
            }
        }
    }
};

Pool &pool() {
    static Pool *p = new Pool;  // never destroyed: its threads live until exit
    return *p;
}

}  // namespace

void parallel_for(int T, const std::function<void(int)> &f) {
    if (T <= 1) {
        f(0);
        return;
    }
    Pool &p = pool();
    std::unique_lock<std::mutex> c(p.call, std::try_to_lock);
    if (!c.owns_lock()) {
        std::vector<std::thread> th;
        for (int t = 1; t < T; ++t) th.emplace_back([&f, t] { f(t); });
        f(0);
        for (auto &x : th) x.join();
        return;
    }
    {
        std::lock_guard<std::mutex> l(p.m);
        while ((int)p.workers.size() < T - 1) {
            const int id = (int)p.workers.size() + 1;
            p.workers.emplace_back([&p, id] { p.loop(id); });
            p.workers.back().detach();
        }
        p.job = &f;
        p.njob = T;
        p.pending = T - 1;
        ++p.gen;
    }
    p.wake.notify_all();
    f(0);
    std::unique_lock<std::mutex> l(p.m);
    p.done.wait(l, [&] { return p.pending == 0; });
}

}  // namespace fc
