// Serving: the queue of submitted registrations, their admission and the serving loop that
// advances the admitted ones.  Host code with no device types: the library runs it over its
// device executor (cgdir_runtime.hip) and the CPU tests over a simulated device.
//
// Admission is first in, first out: the request at the head of the queue is admitted once a
// slot is free and the executor can give it memory; while it waits for memory, nothing behind
// it is admitted.  Admitted requests advance in ticks, one iteration of Algorithm A each per
// tick, their launches merged, on lanes (streams); a lane holds at most two ticks in flight.
// The policy decides the lanes:
//   kServeLockstep     every request on lane 0;
//   kServeLanes        while large and small requests are admitted together, the large ones
//                      (at least large_voxels at the finest level) on lane 0 and the small ones
//                      on lane 1, so that a small request does not advance at the pace of a
//                      large one's launches;
//   kServeLanesSerial  as kServeLanes; in addition, while no request waits for admission, the
//                      large requests run one at a time, oldest first, as a serial queue would
//                      run them; while requests wait, every admitted request advances (merged
//                      launches give more registrations per second).
// The lanes are decided again whenever a request joins or leaves.
//
// The executor does the device work.  Every call comes from the serving thread, except
// release(), which may also come from the threads that cancel or stop (under the queue lock,
// for a request that was never admitted):
//   struct Work                      one request's device state, default-constructible
//   bool start()                     set-up of the serving thread; false fails every request
//   int allocate(Work &)             its memory: CGDIR_OK, CGDIR_E_NOMEM (the request waits at
//                                    the head of the queue) or an error (the request fails)
//   void release(Work &)             its memory back (also for a request never allocated)
//   int setup(Work &, int lane)      its set-up work on `lane`, ordered after its inputs
//   void abandon(Work &)             wait for its work in flight (after a failed set-up)
//   void move(Work &, int lane)      its later work on `lane`, ordered after its earlier work
//   bool lane_open(int lane)         the lane exists and has fewer than two ticks in flight
//   int tick(int lane, const std::vector<Work *> &, std::vector<int> &codes)
//                                    one iteration of each request, merged; a failed request's
//                                    code in `codes`; a failure of the whole tick returned
//   bool finished(const Work &)      every iteration issued (or the stopping rule fired)
//   int64_t voxels(const Work &)     finest-level voxels
//   void progress(const Work &, int *level, int *iter, double *last_delta)
//   int emit(Work &, int error)      with no error, the results to the caller's buffers; then a
//                                    completion mark; returns the request's error
//   bool done(Work &, int error, int *code)
//                                    true once the completion mark is reached; *code = the
//                                    request's final result
//   void stop()                      the loop ends: wait for every lane
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cgdir.h"

namespace cgdir {

enum ServePolicy { kServeLockstep = 0, kServeLanes = 1, kServeLanesSerial = 2 };
constexpr int kServeLaneCount = 2;

inline int64_t steady_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

template <class Exec>
class Server {
  public:
    using Work = typename Exec::Work;
    struct Request {
        uint64_t ticket = 0;
        Work work;
        // read by poll and wait, written under the queue lock
        int state = CGDIR_QUEUED;
        int error = CGDIR_OK;  // the final code
        int64_t t_submit = 0, t_admit = 0, t_done = 0;
        int level = 0, iter = 0;
        double last_delta = 0.0;
        // the serving thread's own
        int failure = CGDIR_OK;  // becomes `error` when the request finishes
        int lane = 0;
        bool emitted = false;
    };

    Server(Exec &exec, int max_slots, int policy, int64_t large_voxels, size_t keep_finished)
        : x_(exec), max_slots_(max_slots), policy_(policy), large_(large_voxels), keep_(keep_finished)
    {
    }
    ~Server() { stop(); }
    Server(const Server &) = delete;
    Server &operator=(const Server &) = delete;

    // Queues a request whose work the caller has prepared; starts the serving thread.
    int submit(std::shared_ptr<Request> r, uint64_t *ticket)
    {
        r->t_submit = steady_ns();
        std::lock_guard<std::mutex> lk(mu_);
        if (stopping_) return CGDIR_E_INVAL;
        const uint64_t t = next_ticket_++;
        r->ticket = t;
        reqs_[t] = std::move(r);
        queue_.push_back(t);
        *ticket = t;
        if (!thread_.joinable()) thread_ = std::thread([this] { loop(); });
        cv_.notify_all();
        return CGDIR_OK;
    }

    int poll(uint64_t ticket, cgdir_status *st)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return CGDIR_E_NOTFOUND;
        const Request &r = *it->second;
        st->state = r.state;
        st->error = r.error;
        st->level = r.level;
        st->iter = r.iter;
        st->last_delta = r.last_delta;
        st->t_submit_ns = r.t_submit;
        st->t_admit_ns = r.t_admit;
        st->t_done_ns = r.t_done;
        return CGDIR_OK;
    }

    // Only a queued request can be cancelled.
    int cancel(uint64_t ticket)
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return CGDIR_E_NOTFOUND;
        if (it->second->state != CGDIR_QUEUED) return CGDIR_E_BUSY;
        finish(it->second.get(), CGDIR_E_CANCELLED);
        cv_.notify_all();
        return CGDIR_OK;
    }

    // The request's final error, once it is done, failed or cancelled (timeout_ns < 0: no limit).
    int wait(uint64_t ticket, int64_t timeout_ns)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return CGDIR_E_NOTFOUND;
        const std::shared_ptr<Request> r = it->second;  // alive while this thread sleeps
        auto pred = [&] { return r->state == CGDIR_DONE || r->state == CGDIR_FAILED || r->state == CGDIR_CANCELLED; };
        if (timeout_ns < 0) {
            cv_.wait(lk, pred);
        } else if (!cv_.wait_for(lk, std::chrono::nanoseconds(timeout_ns), pred)) {
            return CGDIR_E_TIMEOUT;
        }
        return r->error;
    }

    // Cancels the queued requests, lets the admitted ones finish and ends the serving thread.
    void stop()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (uint64_t t : queue_) {
                auto it = reqs_.find(t);
                if (it != reqs_.end() && it->second->state == CGDIR_QUEUED) finish(it->second.get(), CGDIR_E_CANCELLED);
            }
            queue_.clear();
            stopping_ = true;
        }
        cv_.notify_all();
        if (thread_.joinable()) thread_.join();
    }

  private:
    // Final state of a request (under mu_); the oldest finished records beyond keep_ are dropped.
    void finish(Request *r, int code)
    {
        x_.release(r->work);
        r->error = code;
        r->state = code == CGDIR_OK ? CGDIR_DONE : (code == CGDIR_E_CANCELLED ? CGDIR_CANCELLED : CGDIR_FAILED);
        r->t_done = steady_ns();
        finished_.push_back(r->ticket);
        while (finished_.size() > keep_) {
            reqs_.erase(finished_.front());
            finished_.pop_front();
        }
    }

    bool live(const Request *r) const { return !r->emitted && r->failure == CGDIR_OK && !x_.finished(r->work); }
    bool large(const Request *r) const { return x_.voxels(r->work) >= large_; }

    void loop()
    {
        const bool device_ok = x_.start();
        std::vector<Request *> active;
        auto mixed = [&]() {
            if (policy_ == kServeLockstep) return false;
            bool any_large = false, any_small = false;
            for (Request *r : active)
                if (live(r)) (large(r) ? any_large : any_small) = true;
            return any_large && any_small;
        };
        auto lane_of = [&](const Request *r, bool split) { return split && !large(r) ? 1 : 0; };
        auto regroup = [&]() {
            const bool split = mixed();
            for (Request *r : active)
                if (live(r) && lane_of(r, split) != r->lane) {
                    r->lane = lane_of(r, split);
                    x_.move(r->work, r->lane);
                }
        };
        for (;;) {
            // admission, in arrival order.  The request leaves the queue under mu_; its set-up
            // runs after mu_ is released, so that poll, submit and cancel never wait for it.
            bool changed = false;
            for (;;) {
                Request *r = nullptr;
                {
                    std::lock_guard<std::mutex> lk(mu_);
                    while (!queue_.empty()) {
                        auto it = reqs_.find(queue_.front());
                        if (it != reqs_.end() && it->second->state == CGDIR_QUEUED) break;
                        queue_.pop_front();  // (cancelled)
                    }
                    if (queue_.empty() || (int)active.size() >= max_slots_) break;
                    r = reqs_.find(queue_.front())->second.get();
                    const int rc = device_ok ? x_.allocate(r->work) : CGDIR_E_HIP;
                    if (rc == CGDIR_E_NOMEM) break;  // the head of the queue waits for memory
                    queue_.pop_front();
                    if (rc != CGDIR_OK) {
                        finish(r, rc);
                        cv_.notify_all();
                        continue;
                    }
                    r->state = CGDIR_RUNNING;
                    r->t_admit = steady_ns();
                }
                active.push_back(r);
                r->lane = lane_of(r, mixed());
                const int rc = x_.setup(r->work, r->lane);
                if (rc != CGDIR_OK) {
                    x_.abandon(r->work);  // set-up work in flight may still use its memory
                    active.pop_back();
                    std::lock_guard<std::mutex> lk(mu_);
                    finish(r, rc);
                    cv_.notify_all();
                    continue;
                }
                changed = true;
            }
            if (active.empty()) {
                std::unique_lock<std::mutex> lk(mu_);
                if (stopping_ && queue_.empty()) break;
                cv_.wait_for(lk, std::chrono::milliseconds(20));  // new work, or memory for the head
                continue;
            }
            bool backlog;  // requests wait for admission: throughput before the order of arrival
            {
                std::lock_guard<std::mutex> lk(mu_);
                backlog = !queue_.empty();
            }
            // the one large request that advances while there is no backlog: the oldest
            const Request *lead = nullptr;
            if (policy_ == kServeLanesSerial && !backlog)
                for (Request *r : active)
                    if (live(r) && large(r)) {
                        lead = r;
                        break;
                    }
            if (changed) regroup();
            // one tick on every lane that has running requests and room for it
            bool issued = false, ended = false;
            for (int l = 0; l < kServeLaneCount; ++l) {
                if (!x_.lane_open(l)) continue;
                std::vector<Work *> tw;
                std::vector<Request *> tr;
                for (Request *r : active)
                    if (live(r) && r->lane == l && !(lead && large(r) && r != lead)) {
                        tw.push_back(&r->work);
                        tr.push_back(r);
                    }
                if (tw.empty()) continue;
                std::vector<int> codes(tw.size(), CGDIR_OK);
                const int rc = x_.tick(l, tw, codes);
                for (size_t i = 0; i < tr.size(); ++i)
                    if (rc != CGDIR_OK || codes[i] != CGDIR_OK) tr[i]->failure = rc != CGDIR_OK ? rc : codes[i];
                issued = true;
            }
            for (Request *r : active)
                if (!r->emitted && (r->failure != CGDIR_OK || x_.finished(r->work))) {
                    r->failure = x_.emit(r->work, r->failure);
                    r->emitted = true;
                    ended = true;
                }
            // progress and completions
            {
                std::lock_guard<std::mutex> lk(mu_);
                for (size_t i = 0; i < active.size();) {
                    Request *r = active[i];
                    x_.progress(r->work, &r->level, &r->iter, &r->last_delta);
                    int code = CGDIR_OK;
                    if (r->emitted && x_.done(r->work, r->failure, &code)) {
                        finish(r, code);
                        active.erase(active.begin() + i);
                        cv_.notify_all();
                        ended = true;
                    } else {
                        ++i;
                    }
                }
            }
            if (ended) regroup();  // a request left: the rest may change lanes
            if (!issued && !ended) std::this_thread::yield();
        }
        x_.stop();
    }

    Exec &x_;
    const int max_slots_;
    const int policy_;
    const int64_t large_;
    const size_t keep_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::thread thread_;
    bool stopping_ = false;
    uint64_t next_ticket_ = 1;
    std::deque<uint64_t> queue_;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> reqs_;
    std::deque<uint64_t> finished_;
};

}  // namespace cgdir
