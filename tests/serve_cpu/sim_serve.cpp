// The serving loop of libcgdir (paper_1301_0970_amd/csrc/cgdir_serve.h) over a simulated
// device, on the CPU.  A tick on a lane takes simulated time in proportion to the voxels of the
// requests it advances and starts when the lane's previous tick has ended; the two lanes run
// side by side.  Every call of the executor is recorded, and each scenario checks the
// scheduler's rules on the record: first-in first-out admission by free slots and memory (no
// request overtakes the head of the queue), slot and memory reuse, the lanes of each policy,
// one large request at a time while nothing waits, cancellation, failures that stay with their
// request, and stop.  The stress scenario drives submit, poll, wait and cancel from several
// threads at once (built with ThreadSanitizer by the test that runs this program).
//
// usage: sim_serve <scenario>; prints "ok <scenario>" and exits 0, or prints what failed.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "cgdir_serve.h"

using cgdir::Server;

namespace {

int g_failures = 0;
#define CHECK(cond, ...)                                                    \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::printf("FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond);     \
            std::printf(__VA_ARGS__);                                       \
            std::printf("\n");                                              \
            ++g_failures;                                                   \
        }                                                                   \
    } while (0)

int64_t now_ns() { return cgdir::steady_ns(); }

struct TickRec {
    int lane;
    std::vector<int> ids;
    int64_t start, end;
};

// The simulated device.  Everything but release() runs on the serving thread; release() may run
// on a cancelling or stopping thread, under the server's queue lock, as may allocate().
struct SimExec {
    struct Work {
        int id = -1;
        int64_t voxels = 0;
        int64_t need = 0;      // memory
        int iters = 1;         // iterations in all
        int fail_at = -1;      // the tick at this iteration fails the request (-1: never)
        int fail_setup = 0;    // set-up returns this code
        // progress
        int done_iters = 0;
        bool finished = false;
        bool allocated = false;
        int lane = -1;
        int64_t lane_end = 0;  // end of its latest work
        int64_t mark = 0;      // completion mark
    };

    int64_t pool = 0, pool_used = 0, pool_peak = 0;  // (under the server's queue lock)
    int allocated_now = 0, allocated_peak = 0;        // (under the server's queue lock)
    double ns_per_voxel = 2.0;
    int64_t tick_ns = 20000;  // fixed cost of a tick
    bool start_ok = true;

    // the record (serving thread only, read after stop)
    int64_t lane_end[cgdir::kServeLaneCount] = {};
    std::deque<int64_t> inflight[cgdir::kServeLaneCount];
    std::vector<TickRec> ticks;
    std::vector<std::pair<int, int>> moves;  // (id, lane)
    std::vector<int> admitted;              // ids in admission order
    std::map<int, int64_t> finished_at;     // id -> simulated completion
    std::atomic<int> released{0};

    bool start() { return start_ok; }
    int allocate(Work &w)
    {
        if (pool_used + w.need > pool) return CGDIR_E_NOMEM;
        pool_used += w.need;
        pool_peak = std::max(pool_peak, pool_used);
        w.allocated = true;
        allocated_peak = std::max(allocated_peak, ++allocated_now);
        admitted.push_back(w.id);
        return CGDIR_OK;
    }
    void release(Work &w)
    {
        if (w.allocated) {
            pool_used -= w.need;
            --allocated_now;
            w.allocated = false;
        }
        released.fetch_add(1);
    }
    int setup(Work &w, int lane)
    {
        w.lane = lane;
        w.lane_end = std::max(now_ns(), lane_end[lane]);
        return w.fail_setup;
    }
    void abandon(Work &) {}
    void move(Work &w, int lane)
    {
        moves.push_back({w.id, lane});
        w.lane = lane;
    }
    bool lane_open(int lane)
    {
        const int64_t t = now_ns();
        while (!inflight[lane].empty() && inflight[lane].front() <= t) inflight[lane].pop_front();
        return inflight[lane].size() < 2;
    }
    int tick(int lane, const std::vector<Work *> &ws, std::vector<int> &codes)
    {
        TickRec rec{lane, {}, 0, 0};
        int64_t start = std::max(now_ns(), lane_end[lane]);
        double vox = 0;
        for (Work *w : ws) {
            start = std::max(start, w->lane_end);  // after the request's earlier work on any lane
            vox += (double)w->voxels;
            rec.ids.push_back(w->id);
            if (w->lane != lane) std::printf("FAIL tick of %d on lane %d, its lane is %d\n", w->id, lane, w->lane), ++g_failures;
        }
        const int64_t end = start + tick_ns + (int64_t)(vox * ns_per_voxel);
        for (size_t i = 0; i < ws.size(); ++i) {
            Work *w = ws[i];
            if (w->done_iters == w->fail_at) {
                codes[i] = CGDIR_E_NONFINITE;
            } else {
                ++w->done_iters;
                w->finished = w->done_iters >= w->iters;
            }
            w->lane_end = end;
        }
        lane_end[lane] = end;
        inflight[lane].push_back(end);
        rec.start = start;
        rec.end = end;
        ticks.push_back(rec);
        return CGDIR_OK;
    }
    bool finished(const Work &w) const { return w.finished; }
    int64_t voxels(const Work &w) const { return w.voxels; }
    void progress(const Work &w, int *level, int *iter, double *last_delta) const
    {
        *level = 0;
        *iter = w.done_iters;
        *last_delta = 0.0;
    }
    int emit(Work &w, int error)
    {
        w.mark = std::max(w.lane_end, now_ns());
        return error;
    }
    bool done(Work &w, int error, int *code)
    {
        if (now_ns() < w.mark) return false;
        finished_at[w.id] = w.mark;
        *code = error;
        return true;
    }
    void stop() {}
};

using Srv = Server<SimExec>;
using Req = Srv::Request;

std::shared_ptr<Req> make(int id, int64_t voxels, int iters, int64_t need = 1)
{
    auto r = std::make_shared<Req>();
    r->work.id = id;
    r->work.voxels = voxels;
    r->work.iters = iters;
    r->work.need = need;
    return r;
}

cgdir_status status(Srv &s, uint64_t t)
{
    cgdir_status st{};
    const int rc = s.poll(t, &st);
    CHECK(rc == CGDIR_OK, "poll(%llu) = %d", (unsigned long long)t, rc);
    return st;
}

// admission in ticket order; at most `slots` admitted at once
void fifo()
{
    SimExec x;
    x.pool = 1 << 30;
    std::vector<uint64_t> t(24);
    std::vector<int64_t> admit(24);
    {
        Srv s(x, 3, cgdir::kServeLanesSerial, 1 << 20, 4096);
        for (int i = 0; i < 24; ++i) CHECK(s.submit(make(i, 1000 + 997 * (i % 7), 3 + i % 5), &t[i]) == CGDIR_OK, "submit");
        for (int i = 0; i < 24; ++i) CHECK(s.wait(t[i], -1) == CGDIR_OK, "wait %d", i);
        for (int i = 0; i < 24; ++i) {
            const cgdir_status st = status(s, t[i]);
            CHECK(st.state == CGDIR_DONE && st.iter == 3 + i % 5, "request %d: state %d iter %d", i, st.state, st.iter);
            CHECK(st.t_submit_ns <= st.t_admit_ns && st.t_admit_ns <= st.t_done_ns, "request %d timestamps", i);
            admit[i] = st.t_admit_ns;
        }
    }
    for (int i = 1; i < 24; ++i) CHECK(admit[i - 1] <= admit[i], "admission out of order at %d", i);
    for (int i = 0; i < 24; ++i) CHECK(x.admitted[i] == i, "admitted[%d] = %d", i, x.admitted[i]);
    CHECK(x.allocated_peak <= 3, "peak admitted %d > 3 slots", x.allocated_peak);
    CHECK(x.allocated_peak == 3, "slots never all used (peak %d)", x.allocated_peak);
    CHECK(x.pool_used == 0 && x.allocated_now == 0, "memory not returned: %lld", (long long)x.pool_used);
}

// the head of the queue waits for memory and nothing overtakes it
void memory()
{
    SimExec x;
    x.pool = 100;
    const int64_t need[] = {60, 30, 30, 60, 10, 100, 5};
    const int n = 7;
    std::vector<uint64_t> t(n);
    {
        Srv s(x, 8, cgdir::kServeLanesSerial, 1 << 20, 4096);
        for (int i = 0; i < n; ++i) CHECK(s.submit(make(i, 2000, 4, need[i]), &t[i]) == CGDIR_OK, "submit");
        for (int i = 0; i < n; ++i) CHECK(s.wait(t[i], -1) == CGDIR_OK, "wait %d", i);
        for (int i = 1; i < n; ++i)
            CHECK(status(s, t[i - 1]).t_admit_ns <= status(s, t[i]).t_admit_ns, "request %d admitted before %d", i, i - 1);
    }
    for (int i = 0; i < n; ++i) CHECK(x.admitted[i] == i, "admitted[%d] = %d", i, x.admitted[i]);
    CHECK(x.pool_peak <= 100, "pool peak %lld > 100", (long long)x.pool_peak);
    CHECK(x.pool_used == 0, "memory not returned");
}

// Scenarios whose checks compare the times of requests that the test submits one after another
// run on a slower simulated device: its ticks then last far longer than a pass of the serving
// loop and the test's own submit calls, also in a ThreadSanitizer build on a loaded machine.
constexpr double kSlowDevice = 20.0;

int64_t first_tick(const SimExec &x, int id)
{
    for (const TickRec &k : x.ticks)
        if (std::find(k.ids.begin(), k.ids.end(), id) != k.ids.end()) return k.start;
    return -1;
}

// kServeLanesSerial: small requests on lane 1 while a large one runs on lane 0; the large ones
// one at a time, oldest first, while nothing waits for admission
void lanes_serial()
{
    SimExec x;
    x.pool = 1 << 30;
    x.ns_per_voxel = kSlowDevice;
    const int64_t large = 100000;
    std::vector<uint64_t> t(5);
    {
        // (the large ones last: once they are admitted nothing waits, and the rule applies)
        Srv s(x, 8, cgdir::kServeLanesSerial, large, 4096);
        CHECK(s.submit(make(2, large / 10, 30), &t[2]) == CGDIR_OK, "submit");
        CHECK(s.submit(make(3, large / 20, 30), &t[3]) == CGDIR_OK, "submit");
        CHECK(s.submit(make(4, large / 5, 30), &t[4]) == CGDIR_OK, "submit");
        CHECK(s.submit(make(0, 4 * large, 12), &t[0]) == CGDIR_OK, "submit");
        CHECK(s.submit(make(1, 2 * large, 12), &t[1]) == CGDIR_OK, "submit");
        for (uint64_t k : t) CHECK(s.wait(k, -1) == CGDIR_OK, "wait");
    }
    for (const TickRec &k : x.ticks) {
        const bool has0 = std::count(k.ids.begin(), k.ids.end(), 0), has1 = std::count(k.ids.begin(), k.ids.end(), 1);
        CHECK(!(has0 && has1), "the two large requests share a tick");
        for (int id : k.ids) {
            if (id <= 1) CHECK(k.lane == 0, "large request %d ticked on lane %d", id, k.lane);
        }
    }
    CHECK(first_tick(x, 1) >= x.finished_at[0], "the second large request started before the first ended");
    // while a large request runs, the small ones tick on lane 1 beside it
    int small_on_1 = 0;
    for (const TickRec &k : x.ticks)
        if (k.lane == 1) ++small_on_1;
    CHECK(small_on_1 > 0, "no tick on lane 1");
    // overlap: some lane-1 tick runs while a lane-0 tick runs
    bool overlap = false;
    for (const TickRec &a : x.ticks)
        for (const TickRec &b : x.ticks)
            if (a.lane == 0 && b.lane == 1 && b.start < a.end && a.start < b.end) overlap = true;
    CHECK(overlap, "the lanes never ran side by side");
    // small requests finish well before the large ones (they do not wait for them)
    for (int id = 2; id <= 4; ++id) CHECK(x.finished_at[id] < x.finished_at[0], "small request %d finished after the large one", id);
}

// with a backlog every admitted request advances, the large ones together
void lanes_backlog()
{
    SimExec x;
    x.pool = 1 << 30;
    const int64_t large = 100000;
    const int n = 10;
    std::vector<uint64_t> t(n);
    {
        Srv s(x, 3, cgdir::kServeLanesSerial, large, 4096);
        for (int i = 0; i < n; ++i) CHECK(s.submit(make(i, 2 * large, 10), &t[i]) == CGDIR_OK, "submit");
        for (uint64_t k : t) CHECK(s.wait(k, -1) == CGDIR_OK, "wait");
    }
    size_t widest = 0;
    for (const TickRec &k : x.ticks) widest = std::max(widest, k.ids.size());
    CHECK(widest == 3, "with a backlog the ticks should merge every admitted request (widest %zu)", widest);
}

// kServeLanes: both large requests advance together (no one-at-a-time rule)
void lanes_all()
{
    SimExec x;
    x.pool = 1 << 30;
    x.ns_per_voxel = kSlowDevice;
    const int64_t large = 100000;
    std::vector<uint64_t> t(3);
    {
        Srv s(x, 8, cgdir::kServeLanes, large, 4096);
        CHECK(s.submit(make(0, 2 * large, 10), &t[0]) == CGDIR_OK, "submit");
        CHECK(s.submit(make(1, 2 * large, 10), &t[1]) == CGDIR_OK, "submit");
        CHECK(s.submit(make(2, large / 10, 10), &t[2]) == CGDIR_OK, "submit");
        for (uint64_t k : t) CHECK(s.wait(k, -1) == CGDIR_OK, "wait");
    }
    bool together = false;
    for (const TickRec &k : x.ticks)
        if (std::count(k.ids.begin(), k.ids.end(), 0) && std::count(k.ids.begin(), k.ids.end(), 1)) together = true;
    CHECK(together, "the large requests never shared a tick");
}

// kServeLockstep: one lane, every admitted request in every tick
void lockstep()
{
    SimExec x;
    x.pool = 1 << 30;
    std::vector<uint64_t> t(4);
    {
        Srv s(x, 8, cgdir::kServeLockstep, 1000, 4096);
        for (int i = 0; i < 4; ++i) CHECK(s.submit(make(i, i == 0 ? 5000 : 50, 8), &t[i]) == CGDIR_OK, "submit");
        for (uint64_t k : t) CHECK(s.wait(k, -1) == CGDIR_OK, "wait");
    }
    for (const TickRec &k : x.ticks) CHECK(k.lane == 0, "lockstep tick on lane %d", k.lane);
    CHECK(x.moves.empty(), "lockstep moved a request");
}

// a request that joins or leaves regroups the others, and a moved request's work stays ordered
void regroup()
{
    SimExec x;
    x.pool = 1 << 30;
    x.ns_per_voxel = kSlowDevice;
    const int64_t large = 100000;
    std::vector<uint64_t> t(2);
    {
        Srv s(x, 8, cgdir::kServeLanesSerial, large, 4096);
        CHECK(s.submit(make(0, large / 10, 200), &t[0]) == CGDIR_OK, "submit");  // small, alone: lane 0
        std::this_thread::sleep_for(std::chrono::milliseconds(1));
        CHECK(s.submit(make(1, 3 * large, 5), &t[1]) == CGDIR_OK, "submit");    // large joins
        for (uint64_t k : t) CHECK(s.wait(k, -1) == CGDIR_OK, "wait");
    }
    bool to1 = false;
    for (auto &m : x.moves)
        if (m.first == 0 && m.second == 1) to1 = true;
    CHECK(to1, "the small request did not move to lane 1 when the large one joined");
    CHECK(!x.moves.empty() && x.moves.back() == std::make_pair(0, 0), "the small request did not return to lane 0 when the large one left");
    // its ticks never overlap each other (ordered across the move)
    int64_t last_end = 0;
    for (const TickRec &k : x.ticks)
        if (std::count(k.ids.begin(), k.ids.end(), 0)) {
            CHECK(k.start >= last_end, "request 0's ticks overlap across lanes");
            last_end = k.end;
        }
}

// cancel a queued request; a running one cannot be cancelled; unknown tickets
void cancel()
{
    SimExec x;
    x.pool = 1 << 30;
    std::vector<uint64_t> t(6);
    {
        Srv s(x, 1, cgdir::kServeLanesSerial, 1 << 20, 4096);
        for (int i = 0; i < 6; ++i) CHECK(s.submit(make(i, 50000, 40), &t[i]) == CGDIR_OK, "submit");
        // wait until the first request runs
        for (int k = 0; k < 2000 && status(s, t[0]).state != CGDIR_RUNNING; ++k)
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        CHECK(status(s, t[0]).state == CGDIR_RUNNING, "first request not running");
        CHECK(s.cancel(t[0]) == CGDIR_E_BUSY, "cancel of a running request");
        CHECK(s.cancel(t[3]) == CGDIR_OK, "cancel of a queued request");
        CHECK(s.cancel(t[3]) == CGDIR_E_BUSY, "second cancel");
        CHECK(s.cancel(987654) == CGDIR_E_NOTFOUND, "unknown ticket");
        cgdir_status st{};
        CHECK(s.poll(987654, &st) == CGDIR_E_NOTFOUND, "poll of an unknown ticket");
        CHECK(s.wait(987654, 0) == CGDIR_E_NOTFOUND, "wait on an unknown ticket");
        CHECK(s.wait(t[3], -1) == CGDIR_E_CANCELLED, "wait on a cancelled request");
        CHECK(s.wait(t[5], 0) == CGDIR_E_TIMEOUT, "zero timeout on a queued request");
        for (int i : {0, 1, 2, 4, 5}) CHECK(s.wait(t[i], -1) == CGDIR_OK, "wait %d", i);
        CHECK(status(s, t[3]).state == CGDIR_CANCELLED, "state of the cancelled request");
    }
    CHECK(std::find(x.admitted.begin(), x.admitted.end(), 3) == x.admitted.end(), "the cancelled request ran");
}

// a failed tick fails its request alone; failed set-up and allocation fail theirs
void failures()
{
    SimExec x;
    x.pool = 1000;
    std::vector<uint64_t> t(5);
    {
        Srv s(x, 4, cgdir::kServeLanesSerial, 1 << 20, 4096);
        auto a = make(0, 3000, 20);
        a->work.fail_at = 7;
        auto b = make(1, 3000, 20);
        b->work.fail_setup = CGDIR_E_HIP;
        auto c = make(2, 3000, 20);
        auto d = make(3, 3000, 20, 2000);  // more than the pool: waits forever at the head...
        CHECK(s.submit(a, &t[0]) == CGDIR_OK, "submit");
        CHECK(s.submit(b, &t[1]) == CGDIR_OK, "submit");
        CHECK(s.submit(c, &t[2]) == CGDIR_OK, "submit");
        CHECK(s.wait(t[0], -1) == CGDIR_E_NONFINITE, "the failing request");
        CHECK(status(s, t[0]).iter == 7, "failed at iteration %d", status(s, t[0]).iter);
        CHECK(s.wait(t[1], -1) == CGDIR_E_HIP, "the failing set-up");
        CHECK(s.wait(t[2], -1) == CGDIR_OK, "the healthy request");
        CHECK(s.submit(d, &t[3]) == CGDIR_OK, "submit");
        CHECK(s.wait(t[3], 20 * 1000 * 1000) == CGDIR_E_TIMEOUT, "...until it is cancelled");
        CHECK(s.cancel(t[3]) == CGDIR_OK, "cancel the waiting head");
        CHECK(s.submit(make(4, 3000, 5), &t[4]) == CGDIR_OK, "submit");
        CHECK(s.wait(t[4], -1) == CGDIR_OK, "a request behind the cancelled head");
    }
    CHECK(x.pool_used == 0 && x.allocated_now == 0, "memory not returned after failures");
    SimExec dead;
    dead.pool = 1 << 30;
    dead.start_ok = false;
    {
        Srv s(dead, 2, cgdir::kServeLanesSerial, 1 << 20, 4096);
        uint64_t k = 0;
        CHECK(s.submit(make(0, 10, 3), &k) == CGDIR_OK, "submit");
        CHECK(s.wait(k, -1) == CGDIR_E_HIP, "a serving thread without a device fails its requests");
    }
}

// stop: queued requests cancelled, admitted ones finished; submit afterwards refused
void stop()
{
    SimExec x;
    x.pool = 1 << 30;
    std::vector<uint64_t> t(6);
    Srv s(x, 2, cgdir::kServeLanesSerial, 1 << 20, 4096);
    for (int i = 0; i < 6; ++i) CHECK(s.submit(make(i, 100000, 30), &t[i]) == CGDIR_OK, "submit");
    for (int k = 0; k < 2000 && status(s, t[1]).state != CGDIR_RUNNING; ++k)
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    s.stop();
    CHECK(status(s, t[0]).state == CGDIR_DONE && status(s, t[1]).state == CGDIR_DONE, "admitted requests not finished");
    for (int i = 2; i < 6; ++i) CHECK(status(s, t[i]).state == CGDIR_CANCELLED, "queued request %d state %d", i, status(s, t[i]).state);
    uint64_t k = 0;
    CHECK(s.submit(make(9, 10, 1), &k) == CGDIR_E_INVAL, "submit after stop");
    CHECK(x.pool_used == 0, "memory not returned at stop");
}

// finished records beyond the limit are dropped, oldest first
void keep()
{
    SimExec x;
    x.pool = 1 << 30;
    std::vector<uint64_t> t(10);
    {
        Srv s(x, 4, cgdir::kServeLanesSerial, 1 << 20, 3);
        for (int i = 0; i < 10; ++i) {
            CHECK(s.submit(make(i, 100, 2), &t[i]) == CGDIR_OK, "submit");
            CHECK(s.wait(t[i], -1) == CGDIR_OK, "wait");
        }
        cgdir_status st{};
        for (int i = 0; i < 7; ++i) CHECK(s.poll(t[i], &st) == CGDIR_E_NOTFOUND, "record %d kept", i);
        for (int i = 7; i < 10; ++i) CHECK(s.poll(t[i], &st) == CGDIR_OK, "record %d dropped", i);
    }
}

// many threads at once: submitters, pollers, waiters with time-outs, a canceller
void stress()
{
    SimExec x;
    x.pool = 400;
    x.tick_ns = 2000;
    x.ns_per_voxel = 0.05;
    const int threads = 4, per = 60;
    std::vector<std::vector<uint64_t>> tk(threads);
    std::atomic<int> cancelled{0}, done{0}, failed{0};
    {
        Srv s(x, 5, cgdir::kServeLanesSerial, 40000, 100000);
        std::vector<std::thread> th;
        std::mutex tmu;
        std::vector<uint64_t> all;
        for (int w = 0; w < threads; ++w)
            th.emplace_back([&, w] {
                std::mt19937 rng(1234 + w);
                for (int i = 0; i < per; ++i) {
                    const int id = w * per + i;
                    auto r = make(id, 1000 + (int64_t)(rng() % 80000), 1 + (int)(rng() % 12), 10 + (int64_t)(rng() % 150));
                    if (rng() % 4 == 0) r->work.fail_at = (int)(rng() % 3);
                    uint64_t t = 0;
                    if (s.submit(r, &t) != CGDIR_OK) {
                        std::printf("FAIL submit from thread %d\n", w);
                        ++g_failures;
                        continue;
                    }
                    tk[w].push_back(t);
                    {
                        std::lock_guard<std::mutex> g(tmu);
                        all.push_back(t);
                    }
                    if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
                }
            });
        std::atomic<bool> quit{false};
        std::thread poller([&] {
            std::mt19937 rng(99);
            while (!quit.load()) {
                uint64_t t = 0;
                {
                    std::lock_guard<std::mutex> g(tmu);
                    if (!all.empty()) t = all[rng() % all.size()];
                }
                cgdir_status st{};
                if (t) (void)s.poll(t, &st);
                std::this_thread::yield();
            }
        });
        std::thread sweeper([&] {  // polls every ticket in turn, the running ones among them
            while (!quit.load()) {
                uint64_t t = 0;
                {
                    std::lock_guard<std::mutex> g(tmu);
                    t = all.size();
                }
                cgdir_status st{};
                for (uint64_t k = 1; k <= t; ++k) (void)s.poll(k, &st);
            }
        });
        std::thread canceller([&] {
            std::mt19937 rng(7);
            while (!quit.load()) {
                uint64_t t = 0;
                {
                    std::lock_guard<std::mutex> g(tmu);
                    if (!all.empty()) t = all[rng() % all.size()];
                }
                if (t && rng() % 5 == 0) (void)s.cancel(t);
                std::this_thread::sleep_for(std::chrono::microseconds(150));
            }
        });
        for (std::thread &x2 : th) x2.join();
        std::vector<std::thread> waiters;
        for (int w = 0; w < threads; ++w)
            waiters.emplace_back([&, w] {
                for (uint64_t t : tk[w]) {
                    int rc;
                    while ((rc = s.wait(t, 2 * 1000 * 1000)) == CGDIR_E_TIMEOUT) {
                    }
                    if (rc == CGDIR_OK) ++done;
                    else if (rc == CGDIR_E_CANCELLED) ++cancelled;
                    else if (rc == CGDIR_E_NONFINITE) ++failed;
                    else {
                        std::printf("FAIL wait returned %d\n", rc);
                        ++g_failures;
                    }
                }
            });
        for (std::thread &x2 : waiters) x2.join();
        quit.store(true);
        poller.join();
        sweeper.join();
        canceller.join();
    }
    CHECK(done + cancelled + failed == threads * per, "%d + %d + %d requests accounted for", done.load(), cancelled.load(), failed.load());
    CHECK(done > 0 && failed > 0, "done %d failed %d", done.load(), failed.load());
    CHECK(x.pool_peak <= 400, "pool peak %lld", (long long)x.pool_peak);
    CHECK(x.allocated_peak <= 5, "admitted peak %d", x.allocated_peak);
    CHECK(x.pool_used == 0 && x.allocated_now == 0, "memory not returned");
    CHECK(x.released.load() == threads * per, "released %d of %d", x.released.load(), threads * per);
}

}  // namespace

int main(int argc, char **argv)
{
    const std::map<std::string, void (*)()> scenarios = {
        {"fifo", fifo},         {"memory", memory}, {"lanes_serial", lanes_serial}, {"lanes_backlog", lanes_backlog},
        {"lanes_all", lanes_all}, {"lockstep", lockstep}, {"regroup", regroup},     {"cancel", cancel},
        {"failures", failures}, {"stop", stop},     {"keep", keep},                 {"stress", stress}};
    if (argc != 2 || !scenarios.count(argv[1])) {
        std::printf("usage: sim_serve <scenario>:");
        for (auto &kv : scenarios) std::printf(" %s", kv.first.c_str());
        std::printf("\n");
        return 2;
    }
    scenarios.at(argv[1])();
    if (g_failures) return 1;
    std::printf("ok %s\n", argv[1]);
    return 0;
}
