// Host runtime of libcgdir: pool sub-allocator, registration driver (Algorithm A:
// pyramid, coarse demons, finest-level CG-DIR loop, stopping rule), batched execution,
// the device side of the serving loop (cgdir_serve.h), and the C-ABI of include/cgdir.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cgdir.h"
#include "cgdir_internal.h"
#include "cgdir_serve.h"

// Device memory of cgdir_register_static: every per-registration buffer of a registration that
// may not allocate.  Each device the library runs on holds its own copy until the process ends;
// host code reaches it only through the address hipGetSymbolAddress returns for that device
// (the array's name in host code is a host-side stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[CGDIR_STATIC_SCRATCH_BYTES];

namespace cgdir {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;                    // guards g_scratch
void *g_scratch[kMaxDevices] = {};          // the device address of `scratch`, per device
std::mutex g_static_mu[kMaxDevices];        // one static registration at a time per device

// The address of `scratch` on `device` (which must be current), looked up once per device.
void *scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p) g_scratch[device] = p;
        else (void)hipGetLastError();
    }
    return g_scratch[device];
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------------ pool sub-allocator
// First-fit over one device buffer; every registration buffer comes from here.
class Pool {
  public:
    void init(char *base, size_t bytes)
    {
        base_ = base;
        size_ = bytes;
        free_.clear();
        used_.clear();
        if (bytes) free_[0] = bytes;
    }
    void *alloc(size_t bytes)
    {
        std::lock_guard<std::mutex> g(mu_);
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                size_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > bytes) free_[off + bytes] = sz - bytes;
                used_[off] = bytes;
                in_use_ += bytes;
                return base_ + off;
            }
        }
        return nullptr;
    }
    void release(void *p)
    {
        if (!p) return;
        std::lock_guard<std::mutex> g(mu_);
        size_t off = (char *)p - base_;
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t sz = u->second;
        used_.erase(u);
        in_use_ -= sz;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + sz == nx->first) {  // merge with the next block
            sz += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {  // merge with the previous block
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += sz;
                return;
            }
        }
        free_[off] = sz;
    }
    size_t size() const { return size_; }
    size_t in_use()
    {
        std::lock_guard<std::mutex> g(mu_);
        return in_use_;
    }

  private:
    std::mutex mu_;
    char *base_ = nullptr;
    size_t size_ = 0;
    size_t in_use_ = 0;
    std::map<size_t, size_t> free_;
    std::unordered_map<size_t, size_t> used_;
};

// ------------------------------------------------------------------ derived parameters

int gauss_radius(double sigma) { return sigma > 0.0 ? (int)std::ceil(3.0 * sigma) : 0; }

// sampled Gaussian of radius ceil(3 sigma), normalised to sum 1 (computed in double)
void gauss_taps(double sigma, float *w)
{
    const int R = gauss_radius(sigma);
    for (int m = 0; m <= kMaxRadius; ++m) w[m] = 0.f;
    if (R == 0) {
        w[0] = 1.f;
        return;
    }
    double t[kMaxRadius + 1], sum = 0.0;
    for (int m = 0; m <= R; ++m) {
        t[m] = std::exp(-(double)(m * m) / (2.0 * (double)sigma * (double)sigma));
        sum += m == 0 ? t[m] : 2.0 * t[m];
    }
    for (int m = 0; m <= R; ++m) w[m] = (float)(t[m] / sum);
}

Dims level_dims(Dims d0, int l)
{
    Dims d = d0;
    for (int i = 0; i < l; ++i) {
        d.nx = (d.nx + 1) / 2;
        d.ny = (d.ny + 1) / 2;
        d.nz = (d.nz + 1) / 2;
    }
    return d;
}

// launch geometry (tile rows, z planes per block) of the iteration kernels
struct Tuning {
    int step_ty = 8, step_tz = 32;
    int smooth_ty = 8, smooth_tz = 32;
};

// CGDIR_TUNE="step_ty,step_tz,smooth_ty,smooth_tz" overrides the launch geometry
Tuning tuning_from_env()
{
    Tuning t;
    const char *e = std::getenv("CGDIR_TUNE");
    if (e) {
        int a, b, c, d;
        if (std::sscanf(e, "%d,%d,%d,%d", &a, &b, &c, &d) == 4) {
            auto ty_ok = [](int v) { return v == 4 || v == 8 || v == 16; };
            if (ty_ok(a) && b >= 1 && ty_ok(c) && d >= 1) t = Tuning{a, b, c, d};
        }
    }
    return t;
}

bool want_delta(const cgdir_params &p) { return p.stop_mode != 0 || p.delta_hist != nullptr; }

size_t footprint_bytes(Dims d0, int k, const cgdir_params &p, bool host_images)
{
    const size_t n0 = (size_t)d0.n();
    size_t b = 0;
    b += 2 * align_up(3 * n0 * sizeof(float));  // u, u_c
    b += align_up(n0 * sizeof(float));          // warped moving image
    for (int l = 1; l < p.levels; ++l) b += 2 * align_up((size_t)level_dims(d0, l).n() * sizeof(float));
    if (host_images) b += 2 * align_up(n0 * sizeof(float));
    if (k > 0) {  // bit-planes, brick occupancy, stencil structure bits, K_i~
        b += 2 * align_up(n0) + align_up((size_t)brick_dims(d0).n());
        b += align_up(n0) + align_up(n0 * sizeof(float));
        for (int l = 1; l < p.levels; ++l)  // bit-planes and occupancy of coarse contour levels
            if ((p.contour_level_mask >> l) & 1u) {
                const Dims dl = level_dims(d0, l);
                b += 2 * align_up((size_t)dl.n()) + align_up((size_t)brick_dims(dl).n());
            }
    }
    if (want_delta(p)) {
        b += align_up(n0);  // UROI
        b += align_up((size_t)metric_parts(d0) * sizeof(float));
        b += align_up((size_t)std::max(p.iters[0], 1) * sizeof(double));
    }
    b += align_up(8192);  // counters, flags, reduction partials
    return b;
}

// ------------------------------------------------------------------ profiling

enum KernelId { K_STEP, K_SMOOTH, K_DELTA, K_RESTRICT, K_PROLONG, K_PACK, K_UROI, K_WARP, K_MISC, K_COUNT };
const char *kKernelNames[K_COUNT] = {"step", "smooth", "delta", "restrict", "prolong",
                                     "pack_masks", "uroi", "warp", "misc"};

// ------------------------------------------------------------------ tile autotuner
// A pair's results do not depend on the tile shape of any kernel, so the first launches of
// each group rotate through candidate shapes, each timed with HIP events on the stream.  One
// timing of a launch varies by a few per cent from the next, so the three fastest candidates
// of that first round are timed twice more, and the group keeps the finalist with the least
// median time per voxel for the rest of the context's life.  A group is (kernel, radius, dims
// of the launch's largest pair, log2 of the launch's voxel count): launches that mix different
// pairs, as served requests join and leave, fall into few groups, while a launch of many small
// pairs is still tuned apart from one small pair alone.  CGDIR_TUNE fixes the shapes instead.
struct TileCfg {
    int ty, tz;
};
// (the small z chunks give coarse pyramid levels enough blocks to fill 256 CUs)
const TileCfg kStepCands[] = {{8, 32}, {8, 16}, {8, 64}, {8, 128}, {16, 16}, {16, 32}, {16, 64}, {16, 128},
                              {4, 32}, {4, 128}, {8, 8}, {4, 8}, {4, 16}, {8, 4}, {4, 4}, {8, 2}, {4, 2}, {8, 1}};
const TileCfg kSmoothCands[] = {{8, 32}, {8, 8}, {8, 16}, {8, 64}, {8, 128}, {16, 16}, {16, 32}, {16, 64},
                                {16, 128}, {4, 16}, {4, 64}, {4, 8}, {8, 4}, {4, 4}, {8, 2}, {4, 2}, {8, 1}};

class Tuner {
  public:
    bool enabled = true;
    TileCfg fixed_step{8, 32}, fixed_smooth{8, 32};
    bool log = false;

    static constexpr int kFinalists = 3, kRepeats = 3;
    static int ncands(bool step)
    {
        return step ? (int)(sizeof(kStepCands) / sizeof(TileCfg)) : (int)(sizeof(kSmoothCands) / sizeof(TileCfg));
    }

    // shape to use for the next launch of group `key`; *measure >= 0 asks the caller to time
    // the launch with events ev[0], ev[1] and hand them back through record().  Candidates for
    // which too_fine() holds are not tried (nor chosen).
    template <class TooFine>
    TileCfg choose(bool step, const std::string &key, int *measure, TooFine &&too_fine)
    {
        *measure = -1;
        const TileCfg *c = step ? kStepCands : kSmoothCands;
        const int nc = ncands(step);
        if (!enabled) return step ? fixed_step : fixed_smooth;
        Entry &e = table_[key];
        if (e.ms.empty()) e.ms.assign(nc, {});
        if (settle_if_measured(key, e)) return c[e.best];
        while (e.next < nc && too_fine(c[e.next])) ++e.next;  // (left untimed: never a finalist
                                                               // while three others are timed)
        if (e.next < nc) {  // first round: every candidate once
            *measure = e.next;
            return c[e.next++];
        }
        if (e.finalists.empty()) {  // the fastest few of the first round (waiting for its timings)
            for (const Pending &p : e.pending) (void)hipEventSynchronize(p.b);
            poll(e);
            std::vector<int> order(nc);
            for (int i = 0; i < nc; ++i) order[i] = i;
            auto first = [&](int x) { return e.ms[x].empty() ? 1e30f : e.ms[x][0]; };  // (untimed: last)
            std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return first(x) < first(y); });
            e.finalists.assign(order.begin(), order.begin() + std::min(kFinalists, nc));
        }
        const int extra = (int)e.finalists.size() * (kRepeats - 1);
        if (e.fnext < extra) {  // the finalists again, in turn
            *measure = e.finalists[e.fnext % e.finalists.size()];
            ++e.fnext;
            return c[*measure];
        }
        return c[e.finalists[0]];
    }
    // the settled shape of a group, else the first candidate: never asks for a timing
    TileCfg settled_or_default(bool step, const std::string &key)
    {
        if (!enabled) return step ? fixed_step : fixed_smooth;
        const TileCfg *c = step ? kStepCands : kSmoothCands;
        auto it = table_.find(key);
        if (it != table_.end() && settle_if_measured(key, it->second)) return c[it->second.best];
        return c[0];
    }
    // settled groups as "<group> <ty> <tz>" lines (groups whose candidates have all been
    // timed settle here too)
    std::string export_text()
    {
        std::string out;
        for (auto &kv : table_) {
            if (!settle_if_measured(kv.first, kv.second)) continue;
            const TileCfg &c = (kv.first[0] == 'U' ? kStepCands : kSmoothCands)[kv.second.best];
            out += kv.first + ' ' + std::to_string(c.ty) + ' ' + std::to_string(c.tz) + '\n';
        }
        return out;
    }
    // the candidate index of shape (ty, tz) for a group's kernel, or -1
    static int candidate(const std::string &key, int ty, int tz)
    {
        if (key.empty() || (key[0] != 'U' && key[0] != 'S')) return -1;
        const bool step = key[0] == 'U';
        const TileCfg *c = step ? kStepCands : kSmoothCands;
        const int nc = step ? (int)(sizeof(kStepCands) / sizeof(TileCfg)) : (int)(sizeof(kSmoothCands) / sizeof(TileCfg));
        for (int i = 0; i < nc; ++i)
            if (c[i].ty == ty && c[i].tz == tz) return i;
        return -1;
    }
    void settle(const std::string &key, int cand)
    {
        Entry &e = table_[key];
        if (e.ms.empty()) e.ms.assign(ncands(key[0] == 'U'), {});
        e.best = cand;
    }
    void record(const std::string &key, int cand, hipEvent_t a, hipEvent_t b, double voxels)
    {
        table_[key].pending.push_back({cand, a, b, voxels > 0.0 ? 1e6 / voxels : 1.0});
    }
    hipEvent_t event()
    {
        if (!spare_.empty()) {
            hipEvent_t e = spare_.back();
            spare_.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void release_all()
    {
        for (auto &kv : table_)
            for (auto &p : kv.second.pending) {
                (void)hipEventSynchronize(p.b);  // (tear-down: an error leaves nothing to do)
                spare_.push_back(p.a);
                spare_.push_back(p.b);
            }
        table_.clear();
        for (hipEvent_t e : spare_) (void)hipEventDestroy(e);
        spare_.clear();
    }

  private:
    struct Pending {
        int cand;
        hipEvent_t a, b;
        double scale;  // to ms per million voxels of the launch
    };
    struct Entry;
    static float median(std::vector<float> v)
    {
        if (v.empty()) return 1e30f;
        std::sort(v.begin(), v.end());
        return v[v.size() / 2];
    }
    // true once the group has a shape: imported, or chosen now that every finalist's timings
    // have landed (the least median time per voxel)
    bool settle_if_measured(const std::string &key, Entry &e)
    {
        if (e.best >= 0) return true;
        if (e.ms.empty() || e.finalists.empty()) return false;
        poll(e);
        // (every repeat asked for has landed; a timing that could not be taken is just absent)
        if (e.fnext < (int)e.finalists.size() * (kRepeats - 1) || !e.pending.empty()) return false;
        const bool step = key[0] == 'U';
        const TileCfg *c = step ? kStepCands : kSmoothCands;
        e.best = e.finalists[0];
        for (int f : e.finalists)
            if (median(e.ms[f]) < median(e.ms[e.best])) e.best = f;
        if (log) {
            std::fprintf(stderr, "cgdir tune %s -> ty %d tz %d (%.5f ms per Mvoxel, median) |", key.c_str(),
                         c[e.best].ty, c[e.best].tz, median(e.ms[e.best]));
            for (size_t i = 0; i < e.ms.size(); ++i) {
                std::fprintf(stderr, " %d,%d:", c[i].ty, c[i].tz);
                for (float m : e.ms[i]) std::fprintf(stderr, "%.5f/", m);
            }
            std::fprintf(stderr, "\n");
        }
        return true;
    }
    struct Entry {
        int next = 0, best = -1, fnext = 0;
        std::vector<std::vector<float>> ms;   // timings of each candidate (ms per Mvoxel)
        std::vector<int> finalists;
        std::vector<Pending> pending;
    };
    void poll(Entry &e)
    {
        for (size_t i = 0; i < e.pending.size();) {
            Pending &p = e.pending[i];
            if (hipEventQuery(p.b) == hipSuccess) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) e.ms[p.cand].push_back((float)(ms * p.scale));
                else e.ms[p.cand].push_back(1e30f);
                spare_.push_back(p.a);
                spare_.push_back(p.b);
                e.pending.erase(e.pending.begin() + i);
            } else {
                ++i;
            }
        }
    }
    std::map<std::string, Entry> table_;
    std::vector<hipEvent_t> spare_;
};

}  // namespace
}  // namespace cgdir

using namespace cgdir;

struct Job;

// pinned host record through which the host follows a job's progress without blocking
struct PinRec {
    int stop;      // finest-level iterations run when the stopping rule fired, else 0
    int pad;
    double delta;  // a recent delta
};

struct cgdir_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // Lanes: two whole-device streams of batched and served work, created with the context.
    // The serving loop puts its large and small requests on separate lanes (cgdir_serve.h); a
    // batch runs its pairs in one lockstep group on lane 0, or with CGDIR_BATCH_LANES=2 its
    // radius groups spread over both lanes (on average no faster, and less repeatable: the
    // autotuner then times launches that share the device with the other lane's).
    hipStream_t lane_full[2] = {nullptr, nullptr};
    int batch_lanes = 1;
    int serve_policy = kServeLanesSerial;
    int64_t large_voxels = int64_t(8) << 20;   // finest-level voxels of a large request
    void *scratch = nullptr;    // this device's static scratch (cgdir_register_static), or null
    PinRec *static_pin = nullptr;  // pinned record of cgdir_register_static
    void *own_pool = nullptr;
    Pool pool;
    int max_slots = 1;
    bool profile = false;
    Tuning tune;
    Tuner tuner;

    // profiling
    std::mutex prof_mu;
    struct Pending {
        int id;
        hipEvent_t a, b;
        double voxels;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare_events;
    // statistics per (kernel, pyramid level); level slot 7 = set-up work
    int64_t launches[K_COUNT * 8] = {};
    double total_ms[K_COUNT * 8] = {};
    double voxels[K_COUNT * 8] = {};

    // serving (created with the context; its thread starts at the first submission)
    struct Serving;
    std::unique_ptr<Serving> serving;
    std::mutex launch_mu;  // keeps each job's launch sequence contiguous on the stream

    // pinned records, allocated in chunks and recycled
    std::mutex pin_mu;
    std::vector<PinRec *> pin_chunks, pin_free;
    PinRec *take_pin()
    {
        std::lock_guard<std::mutex> g(pin_mu);
        if (pin_free.empty()) {
            constexpr int kChunk = 256;
            PinRec *chunk = nullptr;
            if (hipHostMalloc((void **)&chunk, kChunk * sizeof(PinRec), hipHostMallocDefault) != hipSuccess)
                return nullptr;
            pin_chunks.push_back(chunk);
            for (int i = kChunk - 1; i >= 0; --i) pin_free.push_back(chunk + i);
        }
        PinRec *r = pin_free.back();
        pin_free.pop_back();
        *r = PinRec{};
        return r;
    }
    void give_pin(PinRec *r)
    {
        std::lock_guard<std::mutex> g(pin_mu);
        pin_free.push_back(r);
    }
};

namespace cgdir {
namespace {

hipEvent_t take_event(cgdir_ctx *c)
{
    if (!c->spare_events.empty()) {
        hipEvent_t e = c->spare_events.back();
        c->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void drain_profile(cgdir_ctx *c)  // caller holds prof_mu
{
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->launches[p.id] += 1;
            c->total_ms[p.id] += ms;
            c->voxels[p.id] += p.voxels;
        }
        c->spare_events.push_back(p.a);
        c->spare_events.push_back(p.b);
    }
    c->pending.clear();
}

// Runs `fn` (one kernel launch on stream s), bracketed by events on s when profiling;
// `slot` = kernel id * 8 + pyramid level (7 for set-up work).
thread_local bool t_no_events = false;  // set during cgdir_register_static: create no HIP events

template <typename F>
hipError_t timed(cgdir_ctx *c, hipStream_t s, int slot, double vox, F &&fn)
{
    if (!c->profile || t_no_events) return fn();
    std::lock_guard<std::mutex> g(c->prof_mu);
    if (c->pending.size() > 8192) drain_profile(c);
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return fn();
    const bool ra = hipEventRecord(a, s) == hipSuccess;
    hipError_t e = fn();
    const bool rb = hipEventRecord(b, s) == hipSuccess;
    if (ra && rb) {
        c->pending.push_back({slot, a, b, vox});
    } else {  // (an unrecorded pair is not timed)
        c->spare_events.push_back(a);
        c->spare_events.push_back(b);
    }
    return e;
}

#define CG_TRY(expr)                          \
    do {                                      \
        int _rc = (expr);                     \
        if (_rc != CGDIR_OK) return _rc;      \
    } while (0)
#define HIP_TRY(expr)                         \
    do {                                      \
        if ((expr) != hipSuccess) return CGDIR_E_HIP; \
    } while (0)

// ------------------------------------------------------------------ validation

int check_volume(const cgdir_volume *v)
{
    if (!v || !v->data) return CGDIR_E_INVAL;
    if (v->where != CGDIR_HOST && v->where != CGDIR_DEVICE) return CGDIR_E_INVAL;
    if (v->nx < 1 || v->ny < 1 || v->nz < 1 || v->nx > 4096 || v->ny > 4096 || v->nz > 4096)
        return CGDIR_E_INVAL;
    if ((int64_t)v->nx * v->ny * v->nz > (int64_t(1) << 30)) return CGDIR_E_INVAL;
    return CGDIR_OK;
}

int check_params(const cgdir_params &p, int k)
{
    if (p.levels < 1 || p.levels > CGDIR_MAX_LEVELS) return CGDIR_E_INVAL;
    for (int l = 0; l < p.levels; ++l)
        if (p.iters[l] < 0) return CGDIR_E_INVAL;
    if (p.contour_level_mask >> p.levels) return CGDIR_E_INVAL;  // a bit for a level that does not exist
    const bool voxel_units = p.spacing[0] == 0.f && p.spacing[1] == 0.f && p.spacing[2] == 0.f;
    if (!voxel_units) {
        for (int a = 0; a < 3; ++a)
            if (!(p.spacing[a] > 0.f) || !std::isfinite(p.spacing[a])) return CGDIR_E_INVAL;
    }
    const float sig[3] = {p.sigma_fluid, p.sigma_diff, p.restrict_sigma};
    for (int q = 0; q < 3; ++q) {
        if (!(sig[q] >= 0.f) || !std::isfinite(sig[q])) return CGDIR_E_INVAL;
        // the finest level has the most voxels per unit length: the largest radius
        for (int a = 0; a < 3; ++a) {
            const double h = (voxel_units || q == 2) ? 1.0 : (double)p.spacing[a];
            if (gauss_radius((double)sig[q] / h) > kMaxRadius) return CGDIR_E_INVAL;
        }
    }
    for (int i = 0; i < k; ++i) {
        if (!(p.lambda[i] >= 0.f) || !std::isfinite(p.lambda[i])) return CGDIR_E_INVAL;
        if (p.sign[i] < -1 || p.sign[i] > 1) return CGDIR_E_INVAL;
    }
    if (!std::isfinite(p.intensity_offset)) return CGDIR_E_INVAL;
    if (p.stop_mode != 0 && p.stop_mode != 1) return CGDIR_E_INVAL;
    if (p.stop_window < 1 || !(p.norm_range > 0.f)) return CGDIR_E_INVAL;
    for (int a = 0; a < 3; ++a)
        if (p.uroi_margin[a] < 0 || p.uroi_margin[a] > kMaxUroiMargin) return CGDIR_E_INVAL;
    if (p.initial_dvf) {
        if (p.levels != 1) return CGDIR_E_INVAL;
        if (p.initial_dvf_where != CGDIR_HOST && p.initial_dvf_where != CGDIR_DEVICE) return CGDIR_E_INVAL;
    }
    return CGDIR_OK;
}

int check_masks(const cgdir_masks *m, int *k)
{
    if (!m) {
        *k = 0;
        return CGDIR_OK;
    }
    if (m->k < 0 || m->k > CGDIR_MAX_STRUCTS) return CGDIR_E_INVAL;
    if (m->k > 0) {
        if (!m->planes || (m->where != CGDIR_HOST && m->where != CGDIR_DEVICE)) return CGDIR_E_INVAL;
        for (int i = 0; i < m->k; ++i)
            if (!m->planes[i]) return CGDIR_E_INVAL;
    }
    *k = m->k;
    return CGDIR_OK;
}

int check_request(const cgdir_request &r)
{
    CG_TRY(check_volume(&r.target));
    CG_TRY(check_volume(&r.moving));
    if (r.target.nx != r.moving.nx || r.target.ny != r.moving.ny || r.target.nz != r.moving.nz)
        return CGDIR_E_INVAL;
    int kt = 0, km = 0;
    CG_TRY(check_masks(&r.target_masks, &kt));
    CG_TRY(check_masks(&r.moving_masks, &km));
    if (kt != km) return CGDIR_E_INVAL;
    CG_TRY(check_params(r.params, kt));
    if (!r.dvf_out || (r.dvf_where != CGDIR_HOST && r.dvf_where != CGDIR_DEVICE)) return CGDIR_E_INVAL;
    return CGDIR_OK;
}

}  // namespace
}  // namespace cgdir

// ------------------------------------------------------------------ one registration

struct Job {
    cgdir_ctx *ctx = nullptr;
    hipStream_t st = nullptr;     // the stream of the job's device work (the context's, or a
                                  // lane's when batched or served)
    cgdir_request req{};
    const uint8_t *tplanes[CGDIR_MAX_STRUCTS] = {};
    const uint8_t *mplanes[CGDIR_MAX_STRUCTS] = {};
    int k = 0;
    int L = 1;
    Dims d0{};
    bool host_images = false;
    bool delta_on = false;
    float lam[kMaxStructs] = {}, hs[kMaxStructs] = {};
    int sign[kMaxStructs] = {};
    // Gaussians per level and axis (sigma / voxel size of the level, or sigma in voxels), and
    // each level's launch radius (the largest of the three axes)
    float wf[CGDIR_MAX_LEVELS][3][kMaxRadius + 1], wd[CGDIR_MAX_LEVELS][3][kMaxRadius + 1];
    float wr[kMaxRadius + 1];
    int Rf[CGDIR_MAX_LEVELS] = {}, Rd[CGDIR_MAX_LEVELS] = {}, Rr = 0;
    float gs[CGDIR_MAX_LEVELS][3];   // 0.5 / voxel size per level and axis

    std::vector<void *> allocs;
    const float *I0[CGDIR_MAX_LEVELS] = {}, *T0[CGDIR_MAX_LEVELS] = {};
    uint8_t *mbits = nullptr, *tbits = nullptr, *uroi = nullptr, *mocc = nullptr;
    // per level with contour terms: moving and target bit-planes, moving brick occupancy
    // (index 0 = the finest level's mbits, tbits, mocc)
    uint8_t *mbitsL[CGDIR_MAX_LEVELS] = {}, *tbitsL[CGDIR_MAX_LEVELS] = {}, *moccL[CGDIR_MAX_LEVELS] = {};
    float *ubuf = nullptr, *ucbuf = nullptr;
    float *wI0 = nullptr, *Kbuf = nullptr;
    uint8_t *Fbuf = nullptr;
    float *partials = nullptr;
    double *delta_dev = nullptr;
    int64_t *misc_i64 = nullptr;  // [0] UROI count, [1..] reduction partials
    double *misc_f64 = nullptr;
    int *flag = nullptr;
    int *stop_dev = nullptr;      // device: finest-level iterations run when the rule fired
    PinRec *pin = nullptr;        // pinned copies of stop_dev and of a recent delta
    hipEvent_t pin_ev = nullptr;
    bool pin_busy = false;        // a copy into pin is in flight behind pin_ev
    double last_delta = 0.0;
    double *sign_parts = nullptr;

    // progress
    int level = 0;      // current level (coarsest first)
    int iter = 0;       // iterations done at the current level
    bool level_started = false;
    bool finished = false;
    int iters_done0 = 0;

    size_t need() const { return footprint_bytes(d0, k, req.params, host_images); }

    int init(cgdir_ctx *c, const cgdir_request &r)
    {
        ctx = c;
        st = c->stream;
        CG_TRY(check_request(r));
        req = r;
        k = r.target_masks.k;
        if (r.moving_masks.k != k) return CGDIR_E_INVAL;
        for (int i = 0; i < k; ++i) {
            tplanes[i] = r.target_masks.planes[i];
            mplanes[i] = r.moving_masks.planes[i];
        }
        req.target_masks.planes = tplanes;
        req.moving_masks.planes = mplanes;
        d0 = Dims{r.target.nx, r.target.ny, r.target.nz};
        L = r.params.levels;
        host_images = r.target.where == CGDIR_HOST || r.moving.where == CGDIR_HOST;
        delta_on = want_delta(r.params);
        for (int i = 0; i < k; ++i) {
            lam[i] = r.params.lambda[i];
            sign[i] = r.params.sign[i];
        }
        const bool voxel_units =
            r.params.spacing[0] == 0.f && r.params.spacing[1] == 0.f && r.params.spacing[2] == 0.f;
        for (int l = 0; l < L; ++l) {
            Rf[l] = Rd[l] = 0;
            for (int a = 0; a < 3; ++a) {
                const double h = voxel_units ? 1.0 : (double)r.params.spacing[a] * (double)(1 << l);
                const double sf = (double)r.params.sigma_fluid / h, sd = (double)r.params.sigma_diff / h;
                gauss_taps(sf, wf[l][a]);
                gauss_taps(sd, wd[l][a]);
                Rf[l] = std::max(Rf[l], gauss_radius(sf));
                Rd[l] = std::max(Rd[l], gauss_radius(sd));
                gs[l][a] = (float)(0.5 / h);
            }
        }
        gauss_taps(r.params.restrict_sigma, wr);
        Rr = gauss_radius(r.params.restrict_sigma);
        level = L - 1;
        iter = 0;
        return CGDIR_OK;
    }

    // with an arena (cgdir_register_static) buffers are carved from it in order, else from the
    // context pool
    char *arena = nullptr;
    size_t arena_size = 0, arena_used = 0;

    void *take(size_t bytes)
    {
        if (arena) {
            const size_t off = align_up(arena_used), sz = align_up(bytes ? bytes : 1);
            if (off + sz > arena_size) return nullptr;
            arena_used = off + sz;
            return arena + off;
        }
        void *p = ctx->pool.alloc(bytes);
        if (p) allocs.push_back(p);
        return p;
    }

    void release()
    {
        for (void *p : allocs) ctx->pool.release(p);
        allocs.clear();
        arena_used = 0;
        if (pin_ev) {
            if (pin_busy) (void)hipEventSynchronize(pin_ev);  // no copy may land in a recycled record
            (void)hipEventDestroy(pin_ev);
            pin_ev = nullptr;
            pin_busy = false;
        }
        if (pin) {
            ctx->give_pin(pin);
            pin = nullptr;
        }
    }

    int allocate()
    {
        const size_t n0 = (size_t)d0.n();
        ubuf = (float *)take(3 * n0 * sizeof(float));
        ucbuf = (float *)take(3 * n0 * sizeof(float));
        wI0 = (float *)take(n0 * sizeof(float));
        bool ok = ubuf && ucbuf && wI0;
        if (host_images) {
            float *a = (float *)take(n0 * sizeof(float));
            float *b = (float *)take(n0 * sizeof(float));
            I0[0] = a;
            T0[0] = b;
            ok = ok && a && b;
        } else {
            I0[0] = (const float *)req.moving.data;
            T0[0] = (const float *)req.target.data;
        }
        for (int l = 1; l < L; ++l) {
            const size_t nl = (size_t)level_dims(d0, l).n();
            float *a = (float *)take(nl * sizeof(float));
            float *b = (float *)take(nl * sizeof(float));
            I0[l] = a;
            T0[l] = b;
            ok = ok && a && b;
        }
        if (k > 0) {
            mbits = (uint8_t *)take(n0);
            tbits = (uint8_t *)take(n0);
            mocc = (uint8_t *)take((size_t)brick_dims(d0).n());
            Fbuf = (uint8_t *)take(n0);
            Kbuf = (float *)take(n0 * sizeof(float));
            ok = ok && mbits && tbits && mocc && Fbuf && Kbuf;
            mbitsL[0] = mbits;
            tbitsL[0] = tbits;
            moccL[0] = mocc;
            for (int l = 1; l < L; ++l) {
                if (!contour_at(l)) continue;
                const Dims dl = level_dims(d0, l);
                mbitsL[l] = (uint8_t *)take((size_t)dl.n());
                tbitsL[l] = (uint8_t *)take((size_t)dl.n());
                moccL[l] = (uint8_t *)take((size_t)brick_dims(dl).n());
                ok = ok && mbitsL[l] && tbitsL[l] && moccL[l];
            }
        }
        if (delta_on) {
            uroi = (uint8_t *)take(n0);
            partials = (float *)take((size_t)metric_parts(d0) * sizeof(float));
            delta_dev = (double *)take((size_t)std::max(req.params.iters[0], 1) * sizeof(double));
            ok = ok && uroi && partials && delta_dev;
        }
        char *misc = (char *)take(8192);
        ok = ok && misc;
        if (!ok) {
            release();
            return CGDIR_E_NOMEM;
        }
        misc_i64 = (int64_t *)misc;               // [0] count, [8, 264) count partials
        misc_f64 = (double *)(misc + 2304);        // 4 doubles
        flag = (int *)(misc + 2304 + 64);
        stop_dev = (int *)(misc + 2304 + 96);
        sign_parts = (double *)(misc + 4096);      // 128 x 4 doubles
        if (delta_on) {
            pin = ctx->take_pin();
            if (!pin || hipEventCreateWithFlags(&pin_ev, hipEventDisableTiming) != hipSuccess) {
                pin_ev = nullptr;
                release();
                return CGDIR_E_HIP;
            }
        }
        return CGDIR_OK;
    }

    float *comp(float *base, int c) const { return base + (size_t)c * (size_t)d0.n(); }

    // device setup: copies, mask bits, UROI, signs, pyramid, initial field
    int setup()
    {
        hipStream_t s = st;
        const int64_t n0 = d0.n();
        if (host_images) {
            const hipMemcpyKind km = req.moving.where == CGDIR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
            const hipMemcpyKind kt = req.target.where == CGDIR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
            HIP_TRY(hipMemcpyAsync((void *)I0[0], req.moving.data, n0 * sizeof(float), km, s));
            HIP_TRY(hipMemcpyAsync((void *)T0[0], req.target.data, n0 * sizeof(float), kt, s));
        }
        if (k > 0) {
            for (int side = 0; side < 2; ++side) {
                const cgdir_masks &m = side == 0 ? req.moving_masks : req.target_masks;
                uint8_t *bits = side == 0 ? mbits : tbits;
                const uint8_t *planes[kMaxStructs];
                if (m.where == CGDIR_HOST) {  // stage through the (still unused) uc buffer
                    uint8_t *stage = (uint8_t *)ucbuf;
                    for (int i = 0; i < k; ++i) {
                        HIP_TRY(hipMemcpyAsync(stage + (size_t)i * n0, m.planes[i], n0, hipMemcpyHostToDevice, s));
                        planes[i] = stage + (size_t)i * n0;
                    }
                } else {
                    for (int i = 0; i < k; ++i) planes[i] = m.planes[i];
                }
                HIP_TRY(timed(ctx, st, K_PACK * 8 + 7, (double)n0, [&] { return launch_pack_masks(planes, k, n0, bits, s); }));
                if (m.where == CGDIR_HOST) HIP_TRY(hipStreamSynchronize(s));  // staging reused next side
            }
            HIP_TRY(timed(ctx, st, K_PACK * 8 + 7, (double)n0, [&] { return launch_brick_occupancy(mbits, d0, mocc, s); }));
            for (int l = 1; l < L; ++l) {  // coarse levels with contour terms
                if (!contour_at(l)) continue;
                const Dims dl = level_dims(d0, l);
                HIP_TRY(timed(ctx, st, K_PACK * 8 + l, (double)dl.n(), [&] {
                    hipError_t e = launch_level_bits(mbits, d0, l, mbitsL[l], dl, s);
                    if (e == hipSuccess) e = launch_level_bits(tbits, d0, l, tbitsL[l], dl, s);
                    if (e == hipSuccess) e = launch_brick_occupancy(mbitsL[l], dl, moccL[l], s);
                    return e;
                }));
            }
        }
        // the u_c buffer (12 bytes per voxel) is scratch until the first iteration
        uint8_t *rowdist = (uint8_t *)ucbuf + n0;
        if (delta_on) {
            if (k > 0) {
                HIP_TRY(timed(ctx, st, K_UROI * 8 + 7, (double)n0,
                              [&] { return launch_uroi(tbits, d0, req.params.uroi_margin, rowdist, uroi, s); }));
            } else {
                HIP_TRY(hipMemsetAsync(uroi, 1, n0, s));
            }
            int np = 0;
            HIP_TRY(launch_count(uroi, n0, 0xFF, misc_i64 + 8, &np, misc_i64, s));
        }
        bool need_auto = false;
        for (int i = 0; i < k; ++i) need_auto |= sign[i] == 0;
        if (need_auto) {
            uint8_t *dil = (uint8_t *)ucbuf;  // rowdist follows it
            double *parts = sign_parts;
            for (int i = 0; i < k; ++i) {
                if (sign[i] != 0) continue;
                HIP_TRY(launch_dilate_bit(tbits, i, d0, req.params.uroi_margin, rowdist, dil, s));
                int np = 0;
                HIP_TRY(launch_sign_stats(T0[0], tbits, dil, i, n0, parts, &np, misc_f64, s));
                double h[4];
                HIP_TRY(hipMemcpyAsync(h, misc_f64, sizeof(h), hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                sign[i] = (h[1] == 0.0 || h[3] == 0.0) ? 1 : (h[0] / h[1] >= h[2] / h[3] ? 1 : -1);
            }
        }
        for (int i = 0; i < k; ++i) hs[i] = 0.5f * (float)sign[i];
        // pyramid: R(F)(j) = (G * F)(2j), one axis at a time through two scratch volumes
        for (int l = 1; l < L; ++l) {
            const Dims din = level_dims(d0, l - 1);
            Dims dx = din;
            dx.nx = (din.nx + 1) / 2;
            Dims dy = dx;
            dy.ny = (dx.ny + 1) / 2;
            float *t1 = ucbuf;                   // <= n0 floats
            float *t2 = ucbuf + (size_t)n0;      // <= n0 floats
            for (int img = 0; img < 2; ++img) {
                const float *src = img == 0 ? I0[l - 1] : T0[l - 1];
                float *dst = (float *)(img == 0 ? I0[l] : T0[l]);
                HIP_TRY(timed(ctx, st, K_RESTRICT * 8 + l, (double)din.n(), [&] {
                    hipError_t e = launch_restrict_pass(src, t1, din, 0, wr, Rr, s);
                    if (e == hipSuccess) e = launch_restrict_pass(t1, t2, dx, 1, wr, Rr, s);
                    if (e == hipSuccess) e = launch_restrict_pass(t2, dst, dy, 2, wr, Rr, s);
                    return e;
                }));
            }
        }
        // u0 := 0 at the coarsest level, or the given field at the finest
        if (req.params.initial_dvf) {
            const hipMemcpyKind kd = req.params.initial_dvf_where == CGDIR_HOST ? hipMemcpyHostToDevice
                                                                                : hipMemcpyDeviceToDevice;
            HIP_TRY(hipMemcpyAsync(ubuf, req.params.initial_dvf, 3 * n0 * sizeof(float), kd, s));
        } else {
            HIP_TRY(launch_fill(ubuf, 3 * n0, 0.f, s));
        }
        // (fill kernels rather than memset nodes: a caller may capture this work in a graph)
        HIP_TRY(launch_fill((float *)flag, 1, 0.f, s));
        HIP_TRY(launch_fill((float *)stop_dev, 1, 0.f, s));
        return CGDIR_OK;
    }

    bool contour_at(int l) const { return k > 0 && ((req.params.contour_level_mask >> l) & 1u); }

    // the warp of the moving image with this level's field
    WarpArgs warp_args() const
    {
        const Dims d = level_dims(d0, level);
        const bool contour = contour_at(level);
        WarpArgs w{};
        w.I0 = I0[level];
        w.mbits = contour ? mbitsL[level] : nullptr;
        w.mocc = contour ? moccL[level] : nullptr;
        w.wI0 = wI0;
        w.F = contour ? Fbuf : nullptr;
        w.K = contour ? Kbuf : nullptr;
        w.d = d;
        const Dims db = brick_dims(d);
        w.bnx = db.nx;
        w.bny = db.ny;
        w.c0 = req.params.intensity_offset;
        return w;
    }

    // start of a level: prolongation into it (except at the coarsest), then the warp of
    // the moving image with the level's first field
    int begin_level()
    {
        level_started = true;
        const Dims df = level_dims(d0, level);
        if (level < L - 1) {
            const Dims dc = level_dims(d0, level + 1);
            const float *uc[3] = {comp(ubuf, 0), comp(ubuf, 1), comp(ubuf, 2)};
            float *uf[3] = {comp(ucbuf, 0), comp(ucbuf, 1), comp(ucbuf, 2)};
            HIP_TRY(timed(ctx, st, K_PROLONG * 8 + level, (double)df.n(),
                          [&] { return launch_prolong(uc, dc, uf, df, st); }));
            std::swap(ubuf, ucbuf);
        }
        const float *u3[3] = {comp(ubuf, 0), comp(ubuf, 1), comp(ubuf, 2)};
        const WarpArgs w = warp_args();
        HIP_TRY(timed(ctx, st, K_WARP * 8 + level, (double)df.n(), [&] { return launch_warp_init(w, u3, st); }));
        return CGDIR_OK;
    }

    // ---- one iteration of the loop at the current level, as batched-launch descriptors
    bool metric() const { return delta_on && level == 0; }

    // force, fluid smoothing, compose: u -> u_c
    StepArgs step_args() const
    {
        const Dims d = level_dims(d0, level);
        const bool contour = contour_at(level);
        StepArgs sa{};
        sa.wI0 = wI0;
        sa.F = contour ? Fbuf : nullptr;
        sa.K = contour ? Kbuf : nullptr;
        sa.T0 = T0[level];
        sa.tbits = contour ? tbitsL[level] : nullptr;
        sa.uroi = metric() ? uroi : nullptr;
        sa.I0 = I0[level];
        sa.mbits = contour ? mbitsL[level] : nullptr;
        for (int c = 0; c < 3; ++c) {
            sa.u[c] = comp(ubuf, c);
            sa.uc[c] = comp(ucbuf, c);
        }
        sa.partials = metric() ? partials : nullptr;
        sa.d = d;
        sa.k = contour ? k : 0;
        float lam_sum = 0.f;
        sa.neg = 0;
        for (int i = 0; i < kMaxStructs; ++i) {
            sa.lam[i] = i < k ? lam[i] : 0.f;
            if (i < k && hs[i] < 0.f) sa.neg |= 1u << i;
            if (i < sa.k) lam_sum += sa.lam[i];
        }
        sa.far_l1 = 1.f + lam_sum;
        sa.c0 = req.params.intensity_offset;
        sa.inv_norm = 1.0f / req.params.norm_range;
        for (int m = 0; m <= kMaxRadius; ++m) {
            sa.wx[m] = wf[level][0][m];
            sa.wy[m] = wf[level][1][m];
            sa.wz[m] = wf[level][2][m];
        }
        for (int a = 0; a < 3; ++a) {
            sa.gs[a] = gs[level][a];
            sa.gs2[a] = sa.gs[a] * sa.gs[a];
            sa.far_c[a] = 2.f * sa.gs2[a] * sa.far_l1;
        }
        sa.tz = ctx->tune.step_tz;
        sa.stop = delta_on ? stop_dev : nullptr;
        sa.iter = iter;
        return sa;
    }

    DeltaJob delta_job() const
    {
        DeltaJob j;
        j.partials = partials;
        j.nparts = (int)metric_parts(level_dims(d0, level));
        j.n = iter;
        j.count = misc_i64;
        j.hist = delta_dev;
        j.stop = stop_dev;
        j.eps = (double)req.params.stop_eps;
        j.window = req.params.stop_mode ? req.params.stop_window : 0;
        return j;
    }

    // smooth u_c -> u
    SmoothArgs smooth_args() const
    {
        SmoothArgs sb{};
        for (int c = 0; c < 3; ++c) {
            sb.in[c] = comp(ucbuf, c);
            sb.out[c] = comp(ubuf, c);
        }
        sb.d = level_dims(d0, level);
        sb.tz = ctx->tune.smooth_tz;
        for (int m = 0; m <= kMaxRadius; ++m) {
            sb.wx[m] = wd[level][0][m];
            sb.wy[m] = wd[level][1][m];
            sb.wz[m] = wd[level][2][m];
        }
        sb.warp = warp_args();
        sb.stop = delta_on ? stop_dev : nullptr;
        sb.iter = iter;
        return sb;
    }

    int end_level()
    {
        const Dims d = level_dims(d0, level);
        for (int c = 0; c < 3; ++c) HIP_TRY(launch_nonfinite(comp(ubuf, c), d.n(), flag, st));
        return CGDIR_OK;
    }

    // bring the job to a level with an iteration to run (prolongation, empty levels), or
    // mark it finished
    int prepare()
    {
        while (!finished) {
            if (!level_started) CG_TRY(begin_level());
            if (iter < req.params.iters[level]) return CGDIR_OK;
            CG_TRY(end_level());
            if (level == 0) {
                iters_done0 = iter;
                finished = true;
            } else {
                --level;
                iter = 0;
                level_started = false;
            }
        }
        return CGDIR_OK;
    }

    // bookkeeping after the iteration's launches.  The device applies the stopping rule
    // (the delta kernel sets stop_dev and later launches do nothing for the job); every
    // stop_window iterations the host queues a copy of stop_dev and of the latest delta into
    // pinned memory and looks at it once the copy has landed, without ever waiting for it.
    int after_iteration()
    {
        ++iter;
        if (delta_on && level == 0 && pin) {
            if (pin_busy && hipEventQuery(pin_ev) == hipSuccess) {
                pin_busy = false;
                if (pin->stop) {
                    CG_TRY(end_level());
                    iters_done0 = pin->stop;
                    finished = true;
                    return CGDIR_OK;
                }
                last_delta = pin->delta;
            }
            if (!pin_busy && iter % req.params.stop_window == 0) {
                HIP_TRY(hipMemcpyAsync(&pin->stop, stop_dev, sizeof(int), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipMemcpyAsync(&pin->delta, delta_dev + (iter - 1), sizeof(double), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipEventRecord(pin_ev, st));
                pin_busy = true;
            }
        }
        return prepare();
    }

    // copy the result out (asynchronous on the stream)
    int emit()
    {
        const int64_t n0 = d0.n();
        const hipMemcpyKind kd = req.dvf_where == CGDIR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        HIP_TRY(hipMemcpyAsync(req.dvf_out, ubuf, 3 * n0 * sizeof(float), kd, st));
        return CGDIR_OK;
    }

    // after the stream has drained: host-side outputs and the non-finite check
    int conclude()
    {
        if (delta_on) {
            int stopped = 0;
            HIP_TRY(hipMemcpy(&stopped, stop_dev, sizeof(int), hipMemcpyDeviceToHost));
            if (stopped > 0) iters_done0 = stopped;  // the rule fired before the host saw it
            if (iters_done0 > 0)
                HIP_TRY(hipMemcpy(&last_delta, delta_dev + (iters_done0 - 1), sizeof(double), hipMemcpyDeviceToHost));
        }
        if (delta_on && req.params.delta_hist && iters_done0 > 0) {
            HIP_TRY(hipMemcpy(req.params.delta_hist, delta_dev, iters_done0 * sizeof(double), hipMemcpyDeviceToHost));
        }
        if (req.params.iters_done) *req.params.iters_done = iters_done0;
        int bad = 0;
        if (arena && ctx->static_pin) {  // through the context's pinned record: no staging copy
            HIP_TRY(hipMemcpyAsync(&ctx->static_pin->stop, flag, sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            bad = ctx->static_pin->stop;
        } else {
            HIP_TRY(hipMemcpy(&bad, flag, sizeof(int), hipMemcpyDeviceToHost));
        }
        return bad ? CGDIR_E_NONFINITE : CGDIR_OK;
    }
};

// ------------------------------------------------------------------ one tick
// One iteration of every job that has work left, as batched launches: each phase (step,
// metric, smooth) is one launch over the tiles of up to kBatchStep / kBatchSmooth jobs,
// grouped by the radius of the phase's Gaussian.  A job that
// fails stops with its code in `codes`; the others go on.
namespace cgdir {
namespace {

int run_tick(cgdir_ctx *c, hipStream_t s, const std::vector<Job *> &jobs, std::vector<int> &codes,
             bool settled_only = false)
{
    std::vector<int> act;
    for (size_t i = 0; i < jobs.size(); ++i) {
        if (codes[i] != CGDIR_OK || jobs[i]->finished) continue;
        codes[i] = jobs[i]->prepare();
        if (codes[i] == CGDIR_OK && !jobs[i]->finished) act.push_back((int)i);
    }
    if (act.empty()) return CGDIR_OK;
    int lvl = jobs[act[0]]->level;  // profiling slot: the common level, 6 when mixed
    for (int i : act)
        if (jobs[i]->level != lvl) lvl = 6;

    auto shapes_key = [&](char kind, int radius, const int *idx, int n) {
        Dims big{0, 0, 0};
        double total = 0.0;
        for (int q = 0; q < n; ++q) {
            const Dims d = level_dims(jobs[idx[q]]->d0, jobs[idx[q]]->level);
            total += (double)d.n();
            if (d.n() > big.n()) big = d;
        }
        std::string key(1, kind);
        key += std::to_string(radius) + ':' + std::to_string(big.nx) + 'x' + std::to_string(big.ny) + 'x' +
               std::to_string(big.nz) + '/' + std::to_string((int)std::floor(std::log2(std::max(total, 1.0))));
        return key;
    };
    // a launch, timed for the tuner when it asks
    // settled_only: tile shapes the tuner has settled (else its first candidate), no timing
    // events and no profiling events (cgdir_register_static creates no HIP objects)
    // z chunks of fewer than 8 planes recompute their 2R halo planes for few outputs; they pay
    // only where 8-plane chunks leave the device short of blocks (fewer than 4 per CU), so the
    // tuner does not try them elsewhere
    auto pick = [&](bool step, const std::string &key, int *cand, const std::vector<Dims> &dims) {
        if (settled_only) {
            *cand = -1;
            return c->tuner.settled_or_default(step, key);
        }
        return c->tuner.choose(step, key, cand, [&](const TileCfg &t) {
            if (t.tz >= 8) return false;
            int64_t blocks = 0;
            for (const Dims &d : dims) blocks += tile_blocks(d, t.ty, 8);
            return blocks >= 1024;
        });
    };
    auto tuned = [&](bool measure_it, const std::string &key, int cand, double voxels, auto &&fn) -> hipError_t {
        if (!measure_it) return fn();
        hipEvent_t ea = c->tuner.event(), eb = c->tuner.event();
        if (!ea || !eb) return fn();
        // (a pair that failed to record reads as untimeable: the candidate is then never chosen)
        (void)hipEventRecord(ea, s);
        const hipError_t e = fn();
        (void)hipEventRecord(eb, s);
        c->tuner.record(key, cand, ea, eb, voxels);
        return e;
    };

    std::map<int, std::vector<int>> by_rf, by_rd;
    for (int i : act) {
        by_rf[jobs[i]->Rf[jobs[i]->level]].push_back(i);
        by_rd[jobs[i]->Rd[jobs[i]->level]].push_back(i);
    }
    for (auto &g : by_rf) {
        const std::vector<int> &v = g.second;
        for (size_t b = 0; b < v.size(); b += kBatchStep) {
            StepBatch sb{};
            sb.n = (int)std::min<size_t>(kBatchStep, v.size() - b);
            const std::string key = shapes_key('U', g.first, &v[b], sb.n);
            std::vector<Dims> dims;
            for (int q = 0; q < sb.n; ++q) dims.push_back(level_dims(jobs[v[b + q]]->d0, jobs[v[b + q]]->level));
            int cand = -1;
            const TileCfg cfg = pick(true, key, &cand, dims);
            double vox = 0.0;
            for (int q = 0; q < sb.n; ++q) {
                sb.d[q] = jobs[v[b + q]]->step_args();
                sb.d[q].tz = cfg.tz;
                sb.prefix[q + 1] = sb.prefix[q] + tile_blocks(sb.d[q].d, cfg.ty, cfg.tz);
                vox += (double)sb.d[q].d.n();
            }
            if (settled_only) {
                HIP_TRY(launch_step_batch(sb, g.first, cfg.ty, s));
                continue;
            }
            HIP_TRY(timed(c, s, K_STEP * 8 + lvl, vox, [&] {
                return tuned(cand >= 0, key, cand, vox, [&] { return launch_step_batch(sb, g.first, cfg.ty, s); });
            }));
        }
    }
    {
        DeltaBatch db{};
        for (size_t i = 0; i <= act.size(); ++i) {
            if (i < act.size() && jobs[act[i]]->metric()) db.d[db.n++] = jobs[act[i]]->delta_job();
            if (db.n > 0 && (db.n == kBatchDelta || i == act.size())) {
                HIP_TRY(timed(c, s, K_DELTA * 8 + lvl, 0.0, [&] { return launch_delta_batch(db, s); }));
                db.n = 0;
            }
        }
    }
    for (auto &g : by_rd) {
        const std::vector<int> &v = g.second;
        for (size_t b = 0; b < v.size(); b += kBatchSmooth) {
            SmoothBatch sb{};
            sb.n = (int)std::min<size_t>(kBatchSmooth, v.size() - b);
            const std::string key = shapes_key('S', g.first, &v[b], sb.n);
            std::vector<Dims> dims;
            for (int q = 0; q < sb.n; ++q) dims.push_back(level_dims(jobs[v[b + q]]->d0, jobs[v[b + q]]->level));
            int cand = -1;
            const TileCfg cfg = pick(false, key, &cand, dims);
            double vox = 0.0;
            for (int q = 0; q < sb.n; ++q) {
                sb.d[q] = jobs[v[b + q]]->smooth_args();
                sb.d[q].tz = cfg.tz;
                sb.prefix[q + 1] = sb.prefix[q] + tile_blocks(sb.d[q].d, cfg.ty, cfg.tz);
                vox += (double)sb.d[q].d.n();
            }
            if (settled_only) {
                HIP_TRY(launch_smooth_batch(sb, g.first, cfg.ty, s));
                continue;
            }
            HIP_TRY(timed(c, s, K_SMOOTH * 8 + lvl, vox, [&] {
                return tuned(cand >= 0, key, cand, vox, [&] { return launch_smooth_batch(sb, g.first, cfg.ty, s); });
            }));
        }
    }
    for (int i : act) codes[i] = jobs[i]->after_iteration();
    return CGDIR_OK;
}

// Lockstep groups of jobs, each on its own stream: the ticks of one group are ordered on its
// stream, and the groups advance independently, each with at most two ticks queued ahead.
struct LaneWork {
    hipStream_t s = nullptr;
    std::vector<Job *> jobs;
    std::vector<int> codes;
    std::deque<hipEvent_t> inflight;
};

bool lane_has_work(const LaneWork &L)
{
    for (size_t i = 0; i < L.jobs.size(); ++i)
        if (L.codes[i] == CGDIR_OK && !L.jobs[i]->finished) return true;
    return false;
}

// Runs every lane's jobs to completion.  The host issues a tick wherever a lane has fewer than
// two queued and otherwise yields; a failed tick fails the jobs of its lane only.
int drive_lanes(cgdir_ctx *c, std::vector<LaneWork> &lanes)
{
    std::vector<hipEvent_t> spare;
    int rc = CGDIR_OK;
    for (;;) {
        bool any = false, issued = false;
        for (LaneWork &L : lanes) {
            while (!L.inflight.empty() && hipEventQuery(L.inflight.front()) != hipErrorNotReady) {
                spare.push_back(L.inflight.front());  // (a device error surfaces at the final sync)
                L.inflight.pop_front();
            }
            if (!lane_has_work(L)) continue;
            any = true;
            if (L.inflight.size() >= 2) continue;
            const int t = run_tick(c, L.s, L.jobs, L.codes);
            if (t != CGDIR_OK)
                for (size_t i = 0; i < L.jobs.size(); ++i)
                    if (L.codes[i] == CGDIR_OK && !L.jobs[i]->finished) L.codes[i] = t;
            hipEvent_t e = nullptr;
            if (!spare.empty()) {
                e = spare.back();
                spare.pop_back();
            } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                e = nullptr;
                rc = CGDIR_E_HIP;
            }
            if (e && hipEventRecord(e, L.s) == hipSuccess) L.inflight.push_back(e);
            else if (e) spare.push_back(e);
            issued = true;
        }
        if (!any) break;
        if (!issued) std::this_thread::yield();
    }
    for (LaneWork &L : lanes)
        for (hipEvent_t e : L.inflight) {
            (void)hipEventSynchronize(e);
            spare.push_back(e);
        }
    for (hipEvent_t e : spare) (void)hipEventDestroy(e);
    return rc;
}

}  // namespace
}  // namespace cgdir

// ------------------------------------------------------------------ serving

// The device work of the serving loop (cgdir_serve.h): lane l is the context's stream
// lane_full[l].  Events used here belong to the serving thread alone.
namespace cgdir {
namespace {

struct DeviceExec {
    struct Work {
        Job job;
        hipEvent_t ready_ev = nullptr;  // recorded on the context stream at submission: the inputs
                                        // the caller ordered before it are complete past it
        hipEvent_t done_ev = nullptr;   // after the request's last copy (none: its stream is synced)
        ~Work()
        {
            if (ready_ev) (void)hipEventDestroy(ready_ev);
        }
    };
    cgdir_ctx *c;
    std::deque<hipEvent_t> inflight[kServeLaneCount];  // end of each tick in flight
    std::vector<hipEvent_t> spare;

    explicit DeviceExec(cgdir_ctx *ctx) : c(ctx) {}
    hipEvent_t event()
    {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }
    bool start() { return hipSetDevice(c->device) == hipSuccess; }
    int allocate(Work &w) { return w.job.allocate(); }
    void release(Work &w) { w.job.release(); }
    int setup(Work &w, int lane)
    {
        w.job.st = c->lane_full[lane];
        if (w.ready_ev && hipStreamWaitEvent(w.job.st, w.ready_ev, 0) != hipSuccess) return CGDIR_E_HIP;
        std::lock_guard<std::mutex> lg(c->launch_mu);
        return w.job.setup();
    }
    void abandon(Work &w) { (void)hipStreamSynchronize(w.job.st); }
    void move(Work &w, int lane)
    {
        hipStream_t to = c->lane_full[lane];
        if (w.job.st == to) return;
        hipEvent_t e = event();
        const bool ok = e && hipEventRecord(e, w.job.st) == hipSuccess && hipStreamWaitEvent(to, e, 0) == hipSuccess;
        if (!ok) (void)hipStreamSynchronize(w.job.st);  // (ordered the slow way)
        if (e) spare.push_back(e);  // (a wait captures the event's state when it is called)
        w.job.st = to;
    }
    bool lane_open(int lane)
    {
        std::deque<hipEvent_t> &q = inflight[lane];
        while (!q.empty() && hipEventQuery(q.front()) != hipErrorNotReady) {
            spare.push_back(q.front());  // (a device error shows in the completion checks)
            q.pop_front();
        }
        return c->lane_full[lane] && q.size() < 2;
    }
    int tick(int lane, const std::vector<Work *> &ws, std::vector<int> &codes)
    {
        std::vector<Job *> jobs;
        for (Work *w : ws) jobs.push_back(&w->job);
        std::lock_guard<std::mutex> lg(c->launch_mu);
        const int rc = run_tick(c, c->lane_full[lane], jobs, codes);
        hipEvent_t te = event();
        if (te) {
            if (hipEventRecord(te, c->lane_full[lane]) == hipSuccess) inflight[lane].push_back(te);
            else spare.push_back(te);
        }
        return rc;
    }
    bool finished(const Work &w) const { return w.job.finished; }
    int64_t voxels(const Work &w) const { return w.job.d0.n(); }
    void progress(const Work &w, int *level, int *iter, double *last_delta) const
    {
        *level = w.job.level;
        *iter = w.job.iter;
        *last_delta = w.job.last_delta;
    }
    int emit(Work &w, int error)
    {
        std::lock_guard<std::mutex> lg(c->launch_mu);
        if (error == CGDIR_OK) error = w.job.emit();
        w.done_ev = event();
        if (w.done_ev && hipEventRecord(w.done_ev, w.job.st) != hipSuccess) {
            spare.push_back(w.done_ev);  // (completion then found by a stream sync)
            w.done_ev = nullptr;
        }
        return error;
    }
    bool done(Work &w, int error, int *code)
    {
        const hipError_t q = w.done_ev ? hipEventQuery(w.done_ev) : hipSuccess;
        if (q == hipErrorNotReady) return false;
        // no event: wait for its copies; a failed query or sync (a device error) fails the
        // request instead of leaving it pending
        hipError_t e = q;
        if (!w.done_ev) e = hipStreamSynchronize(w.job.st);
        if (e != hipSuccess && error == CGDIR_OK) error = CGDIR_E_HIP;
        *code = error != CGDIR_OK ? error : w.job.conclude();
        if (w.done_ev) spare.push_back(w.done_ev);
        w.done_ev = nullptr;
        return true;
    }
    void stop()
    {
        for (std::deque<hipEvent_t> &q : inflight)
            for (hipEvent_t e : q) {
                (void)hipEventSynchronize(e);
                spare.push_back(e);
            }
        for (std::deque<hipEvent_t> &q : inflight) q.clear();
        for (hipEvent_t e : spare) (void)hipEventDestroy(e);
        spare.clear();
    }
};

}  // namespace
}  // namespace cgdir

struct cgdir_ctx::Serving {
    cgdir::DeviceExec exec;
    cgdir::Server<cgdir::DeviceExec> server;
    explicit Serving(cgdir_ctx *c)
        : exec(c), server(exec, c->max_slots, c->serve_policy, c->large_voxels, CGDIR_KEEP_FINISHED)
    {
    }
};

// ====================================================================== C-ABI

extern "C" {

void cgdir_params_default(cgdir_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->levels = 1;
    for (int l = 0; l < CGDIR_MAX_LEVELS; ++l) p->iters[l] = 100;
    p->contour_level_mask = 1u;
    p->sigma_fluid = 1.f;
    p->sigma_diff = 1.f;
    p->restrict_sigma = 1.f;
    for (int i = 0; i < CGDIR_MAX_STRUCTS; ++i) {
        p->lambda[i] = 1e-3f;
        p->sign[i] = 1;
    }
    p->intensity_offset = 1000.f;
    p->stop_mode = 0;
    p->stop_eps = 1e-4f;
    p->stop_window = 10;
    p->norm_range = 2500.f;
    p->uroi_margin[0] = 5;
    p->uroi_margin[1] = 5;
    p->uroi_margin[2] = 4;
    p->initial_dvf = nullptr;
    p->initial_dvf_where = CGDIR_DEVICE;
    p->delta_hist = nullptr;
    p->iters_done = nullptr;
}

const char *cgdir_strerror(int code)
{
    switch (code) {
    case CGDIR_OK: return "ok";
    case CGDIR_E_INVAL: return "invalid argument";
    case CGDIR_E_NOMEM: return "pool cannot hold the request";
    case CGDIR_E_HIP: return "HIP runtime error";
    case CGDIR_E_BUSY: return "busy";
    case CGDIR_E_NOTFOUND: return "unknown ticket";
    case CGDIR_E_CANCELLED: return "cancelled";
    case CGDIR_E_NONFINITE: return "non-finite field";
    case CGDIR_E_UNIMPL: return "not implemented";
    case CGDIR_E_TIMEOUT: return "timed out";
    case CGDIR_E_SCRATCH: return "the registration does not fit the static scratch of cgdir_register_static";
    default: return "unknown error";
    }
}

size_t cgdir_footprint(int nx, int ny, int nz, int k, const cgdir_params *params)
{
    cgdir_params def;
    if (!params) {
        cgdir_params_default(&def);
        params = &def;
    }
    if (nx < 1 || ny < 1 || nz < 1 || k < 0 || k > CGDIR_MAX_STRUCTS) return 0;
    if (params->levels < 1 || params->levels > CGDIR_MAX_LEVELS) return 0;
    return footprint_bytes(Dims{nx, ny, nz}, k, *params, false);
}

int cgdir_create(cgdir_ctx **out, const cgdir_ctx_desc *desc)
{
    if (!out || !desc || desc->max_slots < 1 || desc->device < 0) return CGDIR_E_INVAL;
    if (!desc->pool && desc->pool_bytes == 0) return CGDIR_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || desc->device >= ndev) return CGDIR_E_HIP;
    if (hipSetDevice(desc->device) != hipSuccess) return CGDIR_E_HIP;
    std::unique_ptr<cgdir_ctx> c(new cgdir_ctx());
    c->device = desc->device;
    c->max_slots = desc->max_slots;
    c->profile = (desc->flags & CGDIR_CTX_PROFILE) != 0;
    c->tune = tuning_from_env();
    c->tuner.enabled = std::getenv("CGDIR_TUNE") == nullptr;
    c->tuner.fixed_step = TileCfg{c->tune.step_ty, c->tune.step_tz};
    c->tuner.fixed_smooth = TileCfg{c->tune.smooth_ty, c->tune.smooth_tz};
    c->tuner.log = std::getenv("CGDIR_TUNE_LOG") != nullptr;
    if (desc->stream) {
        c->stream = (hipStream_t)desc->stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return CGDIR_E_HIP;
        c->own_stream = true;
    }
    auto drop_streams = [&]() {
        for (hipStream_t &ls : c->lane_full)
            if (ls) (void)hipStreamDestroy(ls);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
    };
    for (hipStream_t &ls : c->lane_full)
        if (hipStreamCreateWithFlags(&ls, hipStreamNonBlocking) != hipSuccess) {
            ls = nullptr;
            drop_streams();
            return CGDIR_E_HIP;
        }
    if (const char *e = std::getenv("CGDIR_BATCH_LANES")) c->batch_lanes = std::max(1, std::min(2, std::atoi(e)));
    if (const char *e = std::getenv("CGDIR_SERVE_LARGE")) c->large_voxels = std::max<int64_t>(1, std::atoll(e));
    if (const char *e = std::getenv("CGDIR_SERVE_POLICY")) c->serve_policy = std::max(0, std::min(2, std::atoi(e)));
    void *pool = desc->pool;
    if (!pool) {
        if (hipMalloc(&c->own_pool, desc->pool_bytes) != hipSuccess) {
            drop_streams();
            return CGDIR_E_NOMEM;
        }
        pool = c->own_pool;
    }
    c->pool.init((char *)pool, desc->pool_bytes);
    // set-up of cgdir_register_static (nothing is allocated in that call itself)
    c->scratch = scratch_address(desc->device);
    c->static_pin = c->take_pin();
    c->serving.reset(new cgdir_ctx::Serving(c.get()));
    *out = c.release();
    return CGDIR_OK;
}

int cgdir_destroy(cgdir_ctx *c)
{
    if (!c) return CGDIR_E_INVAL;
    (void)hipSetDevice(c->device);  // (tear-down goes on whatever the device's state)
    if (c->serving) c->serving->server.stop();  // queued requests cancelled, admitted ones finished
    (void)hipStreamSynchronize(c->stream);
    for (hipStream_t ls : c->lane_full)
        if (ls) (void)hipStreamSynchronize(ls);
    {
        std::lock_guard<std::mutex> g(c->prof_mu);
        drain_profile(c);
        for (hipEvent_t e : c->spare_events) (void)hipEventDestroy(e);
        c->spare_events.clear();
    }
    {
        std::lock_guard<std::mutex> lg(c->launch_mu);
        c->tuner.release_all();
    }
    for (PinRec *chunk : c->pin_chunks) (void)hipHostFree(chunk);
    if (c->own_pool) (void)hipFree(c->own_pool);
    c->serving.reset();
    for (hipStream_t ls : c->lane_full)
        if (ls) {
            (void)hipStreamSynchronize(ls);
            (void)hipStreamDestroy(ls);
        }
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return CGDIR_OK;
}

int cgdir_register(cgdir_ctx *c, const cgdir_volume *target, const cgdir_volume *moving,
                   const cgdir_masks *target_masks, const cgdir_masks *moving_masks, const cgdir_params *params,
                   float *dvf_out, int dvf_where)
{
    if (!c || !target || !moving || !params) return CGDIR_E_INVAL;
    cgdir_request r{};
    r.target = *target;
    r.moving = *moving;
    static const cgdir_masks none = {0, nullptr, CGDIR_DEVICE};
    r.target_masks = target_masks ? *target_masks : none;
    r.moving_masks = moving_masks ? *moving_masks : none;
    r.params = *params;
    r.dvf_out = dvf_out;
    r.dvf_where = dvf_where;
    if (hipSetDevice(c->device) != hipSuccess) return CGDIR_E_HIP;
    Job job;
    CG_TRY(job.init(c, r));
    CG_TRY(job.allocate());
    int rc;
    {
        std::lock_guard<std::mutex> lg(c->launch_mu);
        rc = job.setup();
        std::vector<Job *> jobs{&job};
        std::vector<int> codes{rc};
        while (codes[0] == CGDIR_OK && !job.finished) {
            const int t = run_tick(c, c->stream, jobs, codes);
            if (t != CGDIR_OK) codes[0] = t;
        }
        rc = codes[0];
        if (rc == CGDIR_OK) rc = job.emit();
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess && rc == CGDIR_OK) rc = CGDIR_E_HIP;
    if (rc == CGDIR_OK) rc = job.conclude();
    job.release();
    return rc;
}

int cgdir_register_static(cgdir_ctx *c, const cgdir_volume *target, const cgdir_volume *moving,
                          const cgdir_masks *target_masks, const cgdir_masks *moving_masks,
                          const cgdir_params *params, float *dvf_out)
{
    if (!c || !target || !moving || !params || !dvf_out) return CGDIR_E_INVAL;
    // device buffers only (a host buffer would need a staging copy)
    if (target->where != CGDIR_DEVICE || moving->where != CGDIR_DEVICE) return CGDIR_E_INVAL;
    for (const cgdir_masks *m : {target_masks, moving_masks})
        if (m && m->k > 0 && m->where != CGDIR_DEVICE) return CGDIR_E_INVAL;
    if (params->initial_dvf && params->initial_dvf_where != CGDIR_DEVICE) return CGDIR_E_INVAL;
    // what needs pinned host records, events or host copies of device reductions is not here
    if (params->stop_mode != 0 || params->delta_hist) return CGDIR_E_UNIMPL;
    const int k = target_masks ? target_masks->k : 0;
    for (int i = 0; i < k && i < CGDIR_MAX_STRUCTS; ++i)
        if (params->sign[i] == 0) return CGDIR_E_UNIMPL;
    cgdir_request r{};
    r.target = *target;
    r.moving = *moving;
    static const cgdir_masks none = {0, nullptr, CGDIR_DEVICE};
    r.target_masks = target_masks ? *target_masks : none;
    r.moving_masks = moving_masks ? *moving_masks : none;
    r.params = *params;
    r.dvf_out = dvf_out;
    r.dvf_where = CGDIR_DEVICE;
    if (c->device < 0 || c->device >= kMaxDevices || hipSetDevice(c->device) != hipSuccess) return CGDIR_E_HIP;
    if (!c->scratch || !c->static_pin) return CGDIR_E_HIP;  // the set-up at cgdir_create failed
    Job job;
    CG_TRY(job.init(c, r));
    if (job.need() > (size_t)CGDIR_STATIC_SCRATCH_BYTES) return CGDIR_E_SCRATCH;
    std::lock_guard<std::mutex> dev_lock(g_static_mu[c->device]);  // the array is shared per device
    job.arena = (char *)c->scratch;
    job.arena_size = CGDIR_STATIC_SCRATCH_BYTES;
    CG_TRY(job.allocate());  // (carves the arena: no allocation)
    int rc;
    {
        std::lock_guard<std::mutex> lg(c->launch_mu);
        t_no_events = true;
        rc = job.setup();
        std::vector<Job *> jobs{&job};
        std::vector<int> codes{rc};
        while (codes[0] == CGDIR_OK && !job.finished) {
            const int t = run_tick(c, c->stream, jobs, codes, true);
            if (t != CGDIR_OK) codes[0] = t;
        }
        rc = codes[0];
        if (rc == CGDIR_OK) rc = job.emit();
        t_no_events = false;
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess && rc == CGDIR_OK) rc = CGDIR_E_HIP;
    if (rc == CGDIR_OK) rc = job.conclude();
    job.release();
    return rc;
}

int cgdir_register_batch(cgdir_ctx *c, int n, const cgdir_request *reqs, int *status)
{
    if (!c || n < 0 || (n > 0 && !reqs)) return CGDIR_E_INVAL;
    if (hipSetDevice(c->device) != hipSuccess) {
        if (status)
            for (int i = 0; i < n; ++i) status[i] = CGDIR_E_HIP;
        return CGDIR_E_HIP;
    }
    std::vector<std::unique_ptr<Job>> jobs;
    int first = CGDIR_OK;
    std::vector<int> st(n, CGDIR_OK);
    for (int i = 0; i < n; ++i) {
        std::unique_ptr<Job> j(new Job());
        st[i] = j->init(c, reqs[i]);
        if (st[i] == CGDIR_OK) st[i] = j->allocate();
        jobs.push_back(std::move(j));
    }
    for (int i = 0; i < n; ++i)
        if (st[i] == CGDIR_E_NOMEM) {  // all pairs are resident together
            for (auto &j : jobs) j->release();
            if (status)
                for (int q = 0; q < n; ++q) status[q] = st[q] == CGDIR_OK ? CGDIR_E_NOMEM : st[q];
            return CGDIR_E_NOMEM;
        }
    {
        // lanes: the pairs grouped by their Gaussian radii (the launches of one tick are per
        // radius anyway), the groups spread over the two whole-device lane streams, heaviest
        // first onto the lighter lane; with one group and two lanes the pairs themselves are
        // spread that way.  Every lane first waits for the caller's order on the context stream.
        std::map<std::pair<int, int>, std::vector<int>> groups;
        for (int i = 0; i < n; ++i)
            if (st[i] == CGDIR_OK) groups[{jobs[i]->Rf[0], jobs[i]->Rd[0]}].push_back(i);
        const int nl = std::min<int>(c->batch_lanes, std::max<int>(1, n));
        std::vector<std::vector<int>> units;
        if (groups.size() == 1 && nl > 1) {
            for (int i : groups.begin()->second) units.push_back({i});
        } else {
            for (auto &g : groups) units.push_back(g.second);
        }
        auto work = [&](const std::vector<int> &u) {
            double w = 0.0;
            for (int i : u) w += (double)jobs[i]->d0.n();
            return w;
        };
        std::stable_sort(units.begin(), units.end(),
                         [&](const std::vector<int> &a, const std::vector<int> &b) { return work(a) > work(b); });
        std::vector<LaneWork> lanes(nl);
        std::vector<double> load(nl, 0.0);
        std::vector<std::vector<int>> members(nl);
        for (auto &u : units) {
            const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[l] += work(u);
            for (int i : u) members[l].push_back(i);
        }
        std::lock_guard<std::mutex> lg(c->launch_mu);
        hipEvent_t ready = nullptr;
        if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(ready, c->stream) != hipSuccess) {
            if (ready) (void)hipEventDestroy(ready);
            for (auto &j : jobs) j->release();
            if (status)
                for (int i = 0; i < n; ++i) status[i] = CGDIR_E_HIP;
            return CGDIR_E_HIP;
        }
        for (int l = 0; l < nl; ++l) {
            lanes[l].s = c->lane_full[l];
            (void)hipStreamWaitEvent(lanes[l].s, ready, 0);
            for (int i : members[l]) {
                jobs[i]->st = lanes[l].s;
                st[i] = jobs[i]->setup();
                lanes[l].jobs.push_back(jobs[i].get());
                lanes[l].codes.push_back(st[i]);
            }
        }
        (void)hipEventDestroy(ready);  // (the waits captured it)
        if (drive_lanes(c, lanes) != CGDIR_OK) first = CGDIR_E_HIP;
        for (int l = 0; l < nl; ++l)
            for (size_t q = 0; q < members[l].size(); ++q) st[members[l][q]] = lanes[l].codes[q];
        for (int i = 0; i < n; ++i)
            if (st[i] == CGDIR_OK) st[i] = jobs[i]->emit();
    }
    for (hipStream_t ls : c->lane_full)
        if (hipStreamSynchronize(ls) != hipSuccess) first = CGDIR_E_HIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) first = CGDIR_E_HIP;
    for (int i = 0; i < n; ++i) {
        if (st[i] == CGDIR_OK) st[i] = jobs[i]->conclude();
        jobs[i]->release();
        if (first == CGDIR_OK && st[i] != CGDIR_OK) first = st[i];
        if (status) status[i] = st[i];
    }
    return first;
}

int cgdir_warp(cgdir_ctx *c, const cgdir_volume *src, const float *dvf, int mode, void *out)
{
    if (!c || !src || !src->data || !dvf || !out) return CGDIR_E_INVAL;
    if (src->nx < 1 || src->ny < 1 || src->nz < 1 || (int64_t)src->nx * src->ny * src->nz > (int64_t(1) << 30))
        return CGDIR_E_INVAL;
    if (mode != CGDIR_WARP_LINEAR && mode != CGDIR_WARP_MASK) return CGDIR_E_INVAL;
    if (src->where != CGDIR_HOST && src->where != CGDIR_DEVICE) return CGDIR_E_INVAL;
    if (hipSetDevice(c->device) != hipSuccess) return CGDIR_E_HIP;
    const Dims d{src->nx, src->ny, src->nz};
    const int64_t n = d.n();
    const size_t esz = mode == CGDIR_WARP_LINEAR ? sizeof(float) : 1;
    const bool host = src->where == CGDIR_HOST;
    std::vector<void *> tmp;
    auto take = [&](size_t b) {
        void *p = c->pool.alloc(b);
        if (p) tmp.push_back(p);
        return p;
    };
    auto done = [&](int rc) {
        for (void *p : tmp) c->pool.release(p);
        return rc;
    };
    const void *s_dev = src->data;
    const float *u_dev = dvf;
    void *o_dev = out;
    std::lock_guard<std::mutex> lg(c->launch_mu);
    if (host) {
        void *a = take(n * esz), *b = take(3 * n * sizeof(float)), *o = take(n * esz);
        if (!a || !b || !o) return done(CGDIR_E_NOMEM);
        if (hipMemcpyAsync(a, src->data, n * esz, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipMemcpyAsync(b, dvf, 3 * n * sizeof(float), hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return done(CGDIR_E_HIP);
        s_dev = a;
        u_dev = (const float *)b;
        o_dev = o;
    }
    const float *u3[3] = {u_dev, u_dev + n, u_dev + 2 * n};
    hipError_t e = timed(c, c->stream, K_WARP * 8 + 7, (double)n, [&] {
        return mode == CGDIR_WARP_LINEAR ? launch_warp_linear((const float *)s_dev, d, u3, (float *)o_dev, c->stream)
                                         : launch_warp_mask((const uint8_t *)s_dev, d, u3, (uint8_t *)o_dev, c->stream);
    });
    if (e != hipSuccess) return done(CGDIR_E_HIP);
    if (host && hipMemcpyAsync(out, o_dev, n * esz, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return done(CGDIR_E_HIP);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return done(CGDIR_E_HIP);
    return done(CGDIR_OK);
}

// ------------------------------------------------------------------ evaluation (section 2.3)

void cgdir_eval_params_default(cgdir_eval_params *ep)
{
    if (!ep) return;
    ep->spacing[0] = 1.97f;
    ep->spacing[1] = 1.97f;
    ep->spacing[2] = 2.5f;
    ep->opening_radius = 1;
    ep->uroi_margin[0] = 5;
    ep->uroi_margin[1] = 5;
    ep->uroi_margin[2] = 4;
}

namespace cgdir {
namespace {

// scratch of one evaluation call, returned to the pool on every exit
struct Scratch {
    Pool &pool;
    std::vector<void *> held;
    explicit Scratch(Pool &p) : pool(p) {}
    ~Scratch()
    {
        for (void *q : held) pool.release(q);
    }
    void *take(size_t bytes)
    {
        void *q = pool.alloc(std::max<size_t>(bytes, 256));
        if (q) held.push_back(q);
        return q;
    }
};

// block partials of a reduction, added on the host in block order
int host_sums(const double *dev, int nv, double *out, hipStream_t s)
{
    const int nb = eval_red_blocks();
    std::vector<double> h((size_t)nb * nv);
    HIP_TRY(hipMemcpyAsync(h.data(), dev, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int q = 0; q < nv; ++q) out[q] = 0.0;
    for (int b = 0; b < nb; ++b)
        for (int q = 0; q < nv; ++q) out[q] += h[(size_t)b * nv + q];
    return CGDIR_OK;
}

// 95th percentile of sorted values by linear interpolation between order statistics, with
// the interpolation written from whichever end is nearer
double p95_sorted(double lo, double hi, double g)
{
    const double diff = hi - lo;
    return g >= 0.5 ? hi - diff * (1.0 - g) : lo + diff * g;
}

}  // namespace
}  // namespace cgdir

int cgdir_evaluate(cgdir_ctx *c, const cgdir_volume *target, const cgdir_volume *moving,
                   const cgdir_masks *target_masks, const cgdir_masks *moving_masks, const float *dvf,
                   int dvf_where, const cgdir_eval_params *ep, cgdir_eval *out)
{
    if (!c || !dvf || !ep || !out) return CGDIR_E_INVAL;
    CG_TRY(check_volume(target));
    CG_TRY(check_volume(moving));
    if (target->nx != moving->nx || target->ny != moving->ny || target->nz != moving->nz) return CGDIR_E_INVAL;
    int k = 0, km = 0;
    CG_TRY(check_masks(target_masks, &k));
    CG_TRY(check_masks(moving_masks, &km));
    if (k != km) return CGDIR_E_INVAL;
    if (dvf_where != CGDIR_HOST && dvf_where != CGDIR_DEVICE) return CGDIR_E_INVAL;
    for (int a = 0; a < 3; ++a) {
        if (!(ep->spacing[a] > 0.f) || !std::isfinite(ep->spacing[a])) return CGDIR_E_INVAL;
        if (ep->uroi_margin[a] < 0 || ep->uroi_margin[a] > kMaxUroiMargin) return CGDIR_E_INVAL;
    }
    if (ep->opening_radius < 0 || ep->opening_radius > 16) return CGDIR_E_INVAL;

    if (hipSetDevice(c->device) != hipSuccess) return CGDIR_E_HIP;
    const Dims d{target->nx, target->ny, target->nz};
    const int64_t n = d.n();
    const hipStream_t s = c->stream;
    std::lock_guard<std::mutex> lg(c->launch_mu);
    Scratch sc(c->pool);

    // inputs on the device (host inputs are copied once)
    auto dev_copy = [&](const void *src, size_t bytes, bool host) -> const void * {
        if (!host) return src;
        void *q = sc.take(bytes);
        if (q && hipMemcpyAsync(q, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return nullptr;
        return q;
    };
    const float *T0 = (const float *)dev_copy(target->data, n * sizeof(float), target->where == CGDIR_HOST);
    const float *I0 = (const float *)dev_copy(moving->data, n * sizeof(float), moving->where == CGDIR_HOST);
    const float *u = (const float *)dev_copy(dvf, 3 * n * sizeof(float), dvf_where == CGDIR_HOST);
    if (!T0 || !I0 || !u) return CGDIR_E_NOMEM;
    const uint8_t *tplanes[kMaxStructs] = {}, *mplanes[kMaxStructs] = {};
    for (int i = 0; i < k; ++i) {
        tplanes[i] = (const uint8_t *)dev_copy(target_masks->planes[i], n, target_masks->where == CGDIR_HOST);
        mplanes[i] = (const uint8_t *)dev_copy(moving_masks->planes[i], n, moving_masks->where == CGDIR_HOST);
        if (!tplanes[i] || !mplanes[i]) return CGDIR_E_NOMEM;
    }
    const int nb = eval_red_blocks();
    float *wI = (float *)sc.take(n * sizeof(float));
    double *parts = (double *)sc.take((size_t)nb * 8 * sizeof(double));
    uint8_t *tbits = nullptr, *uroi = nullptr, *rowdist = nullptr;
    uint8_t *D = nullptr, *E = nullptr, *O = nullptr, *BD = nullptr, *BT = nullptr;
    if (!wI || !parts) return CGDIR_E_NOMEM;
    if (k > 0) {
        tbits = (uint8_t *)sc.take(n);
        uroi = (uint8_t *)sc.take(n);
        rowdist = (uint8_t *)sc.take(n);
        D = (uint8_t *)sc.take(n);
        E = (uint8_t *)sc.take(n);
        O = (uint8_t *)sc.take(n);
        BD = (uint8_t *)sc.take(n);
        BT = (uint8_t *)sc.take(n);
        if (!tbits || !uroi || !rowdist || !D || !E || !O || !BD || !BT) return CGDIR_E_NOMEM;
    }

    // ---- intensity: deformed moving image against the target, whole volume and UROI
    const float *u3[3] = {u, u + n, u + 2 * n};
    HIP_TRY(launch_warp_linear(I0, d, u3, wI, s));
    if (k > 0) {
        HIP_TRY(launch_pack_masks(tplanes, k, n, tbits, s));
        HIP_TRY(launch_uroi(tbits, d, ep->uroi_margin, rowdist, uroi, s));
    }
    double p1[6], p2[8];
    HIP_TRY(launch_intensity_pass1(wI, T0, uroi, n, parts, s));
    CG_TRY(host_sums(parts, 6, p1, s));
    const double ma = p1[1] / p1[0], mb = p1[2] / p1[0];
    const double ra = p1[3] > 0 ? p1[4] / p1[3] : 0.0, rb = p1[3] > 0 ? p1[5] / p1[3] : 0.0;
    HIP_TRY(launch_intensity_pass2(wI, T0, uroi, n, ma, mb, ra, rb, parts, s));
    CG_TRY(host_sums(parts, 8, p2, s));
    const double nan = std::nan("");
    auto corr = [&](double saa, double sbb, double sab) {
        const double den = std::sqrt(saa * sbb);
        return den > 0 ? sab / den : nan;
    };
    *out = cgdir_eval{};
    out->k = k;
    out->voxels = (int64_t)p1[0];
    out->rms_id = std::sqrt(p2[0] / p1[0]);
    out->cc = corr(p2[1], p2[2], p2[3]);
    out->uroi_voxels = (int64_t)p1[3];
    out->rms_id_uroi = p1[3] > 0 ? std::sqrt(p2[4] / p1[3]) : nan;
    out->cc_uroi = p1[3] > 0 ? corr(p2[5], p2[6], p2[7]) : nan;

    // ---- structures: overlap, propagated contour, surface distances
    size_t sel_bytes = 0;
    HIP_TRY(select_flagged(nullptr, &sel_bytes, BD, n, nullptr, nullptr, s));
    for (int i = 0; i < k; ++i) {
        out->dsc[i] = out->ssd_mean[i] = out->ssd_sd[i] = out->ssd_p95[i] = nan;
        HIP_TRY(launch_warp_mask(mplanes[i], d, u3, D, s));
        double cnt[3];
        HIP_TRY(launch_overlap_counts(D, tbits, i, n, parts, s));
        CG_TRY(host_sums(parts, 3, cnt, s));
        out->deformed_voxels[i] = (int64_t)cnt[0];
        out->target_voxels[i] = (int64_t)cnt[1];
        out->overlap_voxels[i] = (int64_t)cnt[2];
        if (cnt[0] + cnt[1] > 0) out->dsc[i] = 2.0 * cnt[2] / (cnt[0] + cnt[1]);
        // opening: r erosions then r dilations, ping-pong between E and O
        const uint8_t *cur = D;
        for (int r = 0; r < 2 * ep->opening_radius; ++r) {
            uint8_t *dst = (cur == E) ? O : E;
            HIP_TRY(launch_cross(cur, -1, d, r < ep->opening_radius ? 0 : 1, dst, s));
            cur = dst;
        }
        HIP_TRY(launch_cross(cur, -1, d, 2, BD, s));
        HIP_TRY(launch_cross(tbits, i, d, 2, BT, s));
        double nc = 0, ns = 0;
        HIP_TRY(launch_count_nonzero(BD, n, parts, s));
        CG_TRY(host_sums(parts, 1, &nc, s));
        HIP_TRY(launch_count_nonzero(BT, n, parts, s));
        CG_TRY(host_sums(parts, 1, &ns, s));
        out->contour_points[i] = (int64_t)nc;
        out->surface_points[i] = (int64_t)ns;
        if (nc == 0 || ns == 0) continue;
        const int ncp = (int)nc, nsp = (int)ns;
        size_t sort_bytes = 0;
        HIP_TRY(sort_doubles(nullptr, &sort_bytes, nullptr, nullptr, ncp, s));
        Scratch lists(c->pool);
        int *cpts = (int *)lists.take((size_t)ncp * sizeof(int));
        int *spts = (int *)lists.take((size_t)nsp * sizeof(int));
        double *dist = (double *)lists.take((size_t)ncp * sizeof(double));
        double *sorted = (double *)lists.take((size_t)ncp * sizeof(double));
        int *count = (int *)lists.take(sizeof(int));
        void *temp = lists.take(std::max(sel_bytes, sort_bytes));
        if (!cpts || !spts || !dist || !sorted || !count || !temp) return CGDIR_E_NOMEM;
        size_t tb = sel_bytes;
        HIP_TRY(select_flagged(temp, &tb, BD, n, cpts, count, s));
        tb = sel_bytes;
        HIP_TRY(select_flagged(temp, &tb, BT, n, spts, count, s));
        HIP_TRY(launch_ssd(cpts, ncp, spts, nsp, d, ep->spacing, dist, s));
        tb = sort_bytes;
        HIP_TRY(sort_doubles(temp, &tb, dist, sorted, ncp, s));
        double sums[2];
        HIP_TRY(launch_value_sums(sorted, ncp, 0.0, parts, s));
        CG_TRY(host_sums(parts, 2, sums, s));
        const double mean = sums[0] / ncp;
        HIP_TRY(launch_value_sums(sorted, ncp, mean, parts, s));
        CG_TRY(host_sums(parts, 2, sums, s));
        out->ssd_mean[i] = mean;
        out->ssd_sd[i] = std::sqrt(sums[1] / ncp);
        const double h = (double)(ncp - 1) * 0.95;
        const int lo = (int)std::floor(h), hi = std::min(lo + 1, ncp - 1);
        double v[2];
        HIP_TRY(hipMemcpyAsync(&v[0], sorted + lo, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&v[1], sorted + hi, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        out->ssd_p95[i] = p95_sorted(v[0], v[1], h - lo);
    }
    HIP_TRY(hipStreamSynchronize(s));
    return CGDIR_OK;
}

int cgdir_submit(cgdir_ctx *c, const cgdir_request *req, uint64_t *ticket)
{
    if (!c || !req || !ticket) return CGDIR_E_INVAL;
    using Req = Server<DeviceExec>::Request;
    std::shared_ptr<Req> r = std::make_shared<Req>();
    CG_TRY(r->work.job.init(c, *req));
    if (r->work.job.need() > c->pool.size()) return CGDIR_E_NOMEM;
    // the serving loop runs the request on its lane streams after this point of the context stream
    if (hipSetDevice(c->device) != hipSuccess ||
        hipEventCreateWithFlags(&r->work.ready_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(r->work.ready_ev, c->stream) != hipSuccess)
        return CGDIR_E_HIP;
    return c->serving->server.submit(std::move(r), ticket);
}

int cgdir_poll(cgdir_ctx *c, uint64_t ticket, cgdir_status *st)
{
    if (!c || !st) return CGDIR_E_INVAL;
    return c->serving->server.poll(ticket, st);
}

int cgdir_cancel(cgdir_ctx *c, uint64_t ticket)
{
    if (!c) return CGDIR_E_INVAL;
    return c->serving->server.cancel(ticket);
}

int cgdir_wait(cgdir_ctx *c, uint64_t ticket, int64_t timeout_ns)
{
    if (!c) return CGDIR_E_INVAL;
    return c->serving->server.wait(ticket, timeout_ns);
}

int cgdir_tuning_export(cgdir_ctx *c, char *buf, size_t cap, size_t *len)
{
    if (!c || !len || (cap > 0 && !buf)) return CGDIR_E_INVAL;
    std::string text;
    {
        std::lock_guard<std::mutex> lg(c->launch_mu);
        text = c->tuner.export_text();
    }
    *len = text.size() + 1;
    if (cap < *len) return buf ? CGDIR_E_INVAL : CGDIR_OK;
    std::memcpy(buf, text.c_str(), text.size() + 1);
    return CGDIR_OK;
}

int cgdir_tuning_import(cgdir_ctx *c, const char *text)
{
    if (!c || !text) return CGDIR_E_INVAL;
    std::vector<std::pair<std::string, int>> entries;
    const char *p = text;
    while (*p) {
        const char *e = std::strchr(p, '\n');
        const std::string line(p, e ? (size_t)(e - p) : std::strlen(p));
        p = e ? e + 1 : p + line.size();
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;  // blank line
        char key[128];
        int ty = 0, tz = 0, used = 0;
        if (std::sscanf(line.c_str(), "%127s %d %d %n", key, &ty, &tz, &used) != 3 || (size_t)used != line.size())
            return CGDIR_E_INVAL;
        const int cand = Tuner::candidate(key, ty, tz);
        if (cand < 0) return CGDIR_E_INVAL;
        entries.emplace_back(key, cand);
    }
    std::lock_guard<std::mutex> lg(c->launch_mu);
    for (auto &en : entries) c->tuner.settle(en.first, en.second);
    return CGDIR_OK;
}

int cgdir_kernel_stats(cgdir_ctx *c, cgdir_kernel_stat *out, int cap, int reset)
{
    if (!c || (cap > 0 && !out)) return CGDIR_E_INVAL;
    std::lock_guard<std::mutex> g(c->prof_mu);
    drain_profile(c);
    int n = 0;
    for (int i = 0; i < K_COUNT * 8 && n < cap; ++i) {
        if (c->launches[i] == 0) continue;
        std::memset(out[n].name, 0, sizeof(out[n].name));
        if (i % 8 == 7)
            std::snprintf(out[n].name, sizeof(out[n].name), "%s", kKernelNames[i / 8]);
        else
            std::snprintf(out[n].name, sizeof(out[n].name), "%s@L%d", kKernelNames[i / 8], i % 8);
        out[n].launches = c->launches[i];
        out[n].total_ms = c->total_ms[i];
        out[n].voxels = c->voxels[i];
        ++n;
    }
    if (reset)
        for (int i = 0; i < K_COUNT * 8; ++i) {
            c->launches[i] = 0;
            c->total_ms[i] = 0.0;
            c->voxels[i] = 0.0;
        }
    return n;
}

}  // extern "C"
