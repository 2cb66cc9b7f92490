// Host worker threads of a grid handle.  The step runs the solve loops of
// momentum components 1 .. d-1 and the pressure set-up on threads of their
// own (each loop launches kernels and waits for its convergence flags); the
// threads are created once, on the first step that needs them, and then
// wait for their next task instead of being created and joined every step.
#pragma once
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>

namespace chns {

class WorkerPool {
public:
    static constexpr int kWorkers = 3;
    WorkerPool() {
        for (int w = 0; w < kWorkers; ++w) slot_[w].t = std::thread([this, w]() { loop(w); });
    }
    ~WorkerPool() {
        for (int w = 0; w < kWorkers; ++w) {
            {
                std::lock_guard<std::mutex> lk(slot_[w].m);
                slot_[w].stop = true;
            }
            slot_[w].cv.notify_all();
            slot_[w].t.join();
        }
    }
    WorkerPool(const WorkerPool &) = delete;
    WorkerPool &operator=(const WorkerPool &) = delete;
    // Start f on worker w (0 <= w < kWorkers); the worker must be idle.
    void run(int w, std::function<void()> f) {
        {
            std::lock_guard<std::mutex> lk(slot_[w].m);
            slot_[w].task = std::move(f);
            slot_[w].busy = true;
        }
        slot_[w].cv.notify_all();
    }
    // Wait until worker w has finished its task.
    void wait(int w) {
        std::unique_lock<std::mutex> lk(slot_[w].m);
        slot_[w].cv.wait(lk, [&]() { return !slot_[w].busy; });
    }

private:
    struct Slot {
        std::thread t;
        std::mutex m;
        std::condition_variable cv;
        std::function<void()> task;
        bool busy = false, stop = false;
    };
    Slot slot_[kWorkers];
    void loop(int w) {
        Slot &s = slot_[w];
        for (;;) {
            std::function<void()> f;
            {
                std::unique_lock<std::mutex> lk(s.m);
                s.cv.wait(lk, [&]() { return s.stop || s.busy; });
                if (s.busy) f = std::move(s.task);
                else return;   // stop with no task pending
            }
            f();
            {
                std::lock_guard<std::mutex> lk(s.m);
                s.busy = false;
                s.task = nullptr;
            }
            s.cv.notify_all();
        }
    }
};

}  // namespace chns
