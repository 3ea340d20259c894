// Serving loop for a stream of independent mapping jobs (Algorithm 2 per
// job): first-in first-out admission under a fixed device-memory budget, job
// state resident in device memory from admission to retirement, and
// continuous batching: running jobs of one class advance together, one LADMM
// iteration per shared fused launch, joining and leaving at iteration
// boundaries while the others keep running.
//
// Host-side structure:
//   * Slab   - first-fit allocator over one device allocation of the budget;
//              freed ranges coalesce and remember which stream last used them.
//   * Lane   - a HIP stream plus a sequence of fence events; a range freed on
//              one lane is reused on another only after that lane's fence.
//   * Staging- a pinned host ring that feeds every host-to-device upload, so
//              enqueueing never blocks on pageable copies.
//   * Class  - running jobs sharing a fused kernel (precision, padded rank,
//              u K-step bucket, brick shape) and a size band (bytes moved per
//              iteration), with its own round counter, a
//              device descriptor/brick table rebuilt when membership changes,
//              and a lane. Each job's descriptor pair is picked by
//              (round + phase) & 1, the phase being its admission round.

#include "../../include/ssmap.h"
#include "internal.h"
#include "slab.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

using namespace ssmap;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kStagingBytes = (size_t)64 << 20;
constexpr int kFlagSlots = 4096;
constexpr int kServedChecks = 32;       // monitor checks a served job may ask for
constexpr double kBytesPerMs = 4.0e9;     // round-time model: ~4 TB/s sustained
constexpr double kLaunchMs = 0.006;

struct SvFail {
    ssmap_status status;
    std::string msg;
};
[[noreturn]] void sfail(ssmap_status st, const std::string &m) { throw SvFail{st, m}; }

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

using Clock = std::chrono::steady_clock;

struct Lane {
    hipStream_t s = nullptr;
    uint64_t seq = 0, done = 0;
    std::deque<std::pair<uint64_t, hipEvent_t>> pend;
};

// Device images of one (precision, rank, beta) variant of a dictionary.
struct Consts {
    int mode = 0, r = 0, RP = 0;
    void *V = nullptr, *b = nullptr, *Vop = nullptr;
    double *Ur = nullptr, *sig = nullptr, *acoef = nullptr;
    Fence ready;                          // upload fence
};

struct Dict {
    int P = 0, Q = 0, kmin = 0, Qp = 0, nchunk = 0;
    std::vector<double> U, s, V;
    std::map<std::tuple<int, int, uint64_t>, Consts> consts;
};

enum JobState { QUEUED = SSMAP_JOB_QUEUED, RUNNING = SSMAP_JOB_RUNNING, DONE = SSMAP_JOB_DONE };

struct Job {
    int dict = 0;
    Grid g{};
    const void *dM = nullptr;
    void *dF = nullptr;
    double lambda = 0;
    ssmap_steps st{};
    int iters = 0;
    int mode = 0, r = 0, RP = 0;
    double xi = 0, tau = 0;
    size_t bytes = 0, off = 0;
    int cls = -1;
    int64_t r0 = 0;                       // class round of iteration 0
    IterArgs a{};                         // iteration-0 descriptor (z, znew swapped by parity)
    void *z[2] = {nullptr, nullptr};
    int *bad = nullptr;
    int slot = -1;                        // pinned flag slot
    bool retired = false;
    hipEvent_t done_ev = nullptr;
    int state = QUEUED, status = SSMAP_OK;
    double submit_ms = 0, admit_ms = 0, done_ms = 0;
    // monitoring (check_every > 0): U_r^T m, ||m_perp||^2 and the sums of each check
    // (ST_COUNT doubles) in the job's memory; the singular values; the job's bricks
    // in its class's brick table; the checks taken (iterations) and, once done, their sums
    int check_every = 0, nchecks = 0;
    double *t = nullptr, *mperp2 = nullptr, *hist = nullptr;
    const double *sig = nullptr;
    int tile_off = 0, tile_cnt = 0;
    std::vector<int> hist_iter;
    std::vector<double> hist_sums;
    // masked job: the code byte of every voxel (bit 7 inside, bits 0..2 inside face
    // neighbours), on the host and in the job's memory
    std::vector<uint8_t> code;
    uint8_t *dcode = nullptr;
    double dtd = 0;                       // ||D^T D|| of the job's grid (or of its mask's graph)
};

struct Class {
    int mode = 0, RP = 0, rkey = 0;       // rkey: largest rank of the K-step bucket
    int band = 0;                         // size band of the member jobs
    FusedShape shape{16, 1};
    int lane = 0;
    int64_t round = 0;
    std::vector<int64_t> members;
    bool dirty = false;
    IterArgs *djobs = nullptr;
    TileRef *dtiles = nullptr;
    double *dmon = nullptr;                // per-brick (z^{k+1} - z^k)^2 of a monitored round
    size_t cap_jobs = 0, cap_tiles = 0, cap_mon = 0;
    int ntiles = 0;
    int maxchunk = 0;                // largest chunk count among the members
    double model_ms = 0;                  // modelled duration of one round (alone on the GPU)
    double ratio = 1.0;                   // measured / modelled round time (running mean)
    struct Chunk {
        hipEvent_t start, end;
        int64_t rounds;
    };
    std::deque<Chunk> chunks;             // enqueued chunks of rounds, oldest first
};

int bucket_rank(int r) { return r <= 16 ? 16 : r <= 20 ? 20 : r <= 24 ? 24 : 32; }

}  // namespace

struct ssmap_server {
    int device = 0;
    bool poisoned = false;
    std::string err;
    double budget = 0;
    uint8_t *slab_base = nullptr;
    Slab slab;
    int nlanes = 0;
    Lane lanes[kMaxLanes];
    // pinned staging ring
    uint8_t *stage = nullptr;
    size_t stage_head = 0;
    struct Region {
        size_t b, e;
        hipEvent_t ev;
    };
    std::deque<Region> stage_live;
    // pinned non-finite flags, one slot per unfinished job
    int *flags = nullptr;
    // monitored jobs: pinned check sums per slot (kServedChecks x ST_COUNT doubles each)
    // and a partial-sum buffer per lane, both allocated at the first monitored job
    double *hist_pinned = nullptr;
    double *lane_partial[kMaxLanes] = {};
    std::vector<int> free_slots;
    std::vector<hipEvent_t> fence_pool, timing_pool;
    std::vector<void *> dev_allocs;       // consts and tables (freed at destroy)
    std::vector<Dict> dicts;
    std::vector<Job> jobs;
    std::deque<int64_t> queue;
    std::vector<Class> classes;
    // Jobs of the large size band iterate one at a time, in arrival order: two such
    // jobs sharing the GPU would each take about twice as long, so the later one
    // gains nothing while the earlier one finishes late. Admitted large jobs wait
    // here (state resident, projection done) until the running one retires; small
    // and middle jobs keep running beside it.
    std::deque<int64_t> large_wait;
    int64_t large_running = -1;
    hipEvent_t epoch = nullptr;
    Clock::time_point t0;
    ssmap_server_stats stats{};
};

namespace {

std::string g_server_create_error;

void hipx(ssmap_server *sv, hipError_t e, const char *what) {
    if (e != hipSuccess) {
        if (sv) sv->poisoned = true;
        sfail(SSMAP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
}
#define HIPS(sv, call) hipx(sv, (call), #call)

double host_ms(const ssmap_server *sv) {
    return std::chrono::duration<double, std::milli>(Clock::now() - sv->t0).count();
}

hipEvent_t get_event(ssmap_server *sv, bool timing) {
    auto &pool = timing ? sv->timing_pool : sv->fence_pool;
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    HIPS(sv, hipEventCreateWithFlags(&e, timing ? hipEventDefault : hipEventDisableTiming));
    return e;
}
void put_event(ssmap_server *sv, hipEvent_t e, bool timing) {
    (timing ? sv->timing_pool : sv->fence_pool).push_back(e);
}

// true when complete; false when still pending (the not-ready status is cleared)
bool event_done(ssmap_server *sv, hipEvent_t e) {
    const hipError_t q = hipEventQuery(e);
    if (q == hipSuccess) return true;
    if (q == hipErrorNotReady) {
        (void)hipGetLastError();
        return false;
    }
    HIPS(sv, q);
    return false;
}

uint64_t fence_record(ssmap_server *sv, int li) {
    Lane &L = sv->lanes[li];
    hipEvent_t e = get_event(sv, false);
    HIPS(sv, hipEventRecord(e, L.s));
    L.pend.push_back({++L.seq, e});
    return L.seq;
}

void lane_poll(ssmap_server *sv, int li) {
    Lane &L = sv->lanes[li];
    while (!L.pend.empty() && event_done(sv, L.pend.front().second)) {
        L.done = L.pend.front().first;
        put_event(sv, L.pend.front().second, false);
        L.pend.pop_front();
    }
}

// Make lane `dst` wait for the fences of other lanes that are still pending.
void fence_wait(ssmap_server *sv, int dst, const Fence &f) {
    for (int li = 0; li < sv->nlanes; ++li) {
        if (li == dst || f.seq[li] == 0) continue;
        Lane &L = sv->lanes[li];
        if (f.seq[li] <= L.done) continue;
        lane_poll(sv, li);
        if (f.seq[li] <= L.done) continue;
        for (auto &pe : L.pend)
            if (pe.first >= f.seq[li]) {
                HIPS(sv, hipStreamWaitEvent(sv->lanes[dst].s, pe.second, 0));
                break;
            }
    }
}

// Host-to-device copy through the pinned ring, ordered on lane li.
void upload(ssmap_server *sv, int li, void *dst, const void *src, size_t n) {
    if (n == 0) return;
    const size_t m = align_up(n);
    if (m > kStagingBytes) sfail(SSMAP_EINVAL, "upload larger than the staging ring");
    size_t p = sv->stage_head;
    if (p + m > kStagingBytes) p = 0;
    auto overlaps = [&](const ssmap_server::Region &r) { return r.b < p + m && p < r.e; };
    while (std::any_of(sv->stage_live.begin(), sv->stage_live.end(), overlaps)) {
        ssmap_server::Region r = sv->stage_live.front();
        HIPS(sv, hipEventSynchronize(r.ev));
        put_event(sv, r.ev, false);
        sv->stage_live.pop_front();
    }
    std::memcpy(sv->stage + p, src, n);
    HIPS(sv, hipMemcpyAsync(dst, sv->stage + p, n, hipMemcpyHostToDevice, sv->lanes[li].s));
    hipEvent_t e = get_event(sv, false);
    HIPS(sv, hipEventRecord(e, sv->lanes[li].s));
    sv->stage_live.push_back({p, p + m, e});
    sv->stage_head = p + m;
}

void *dev_alloc(ssmap_server *sv, size_t n) {
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, std::max<size_t>(n, kAlign));
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        sfail(SSMAP_ENOMEM, "hipMalloc failed for server tables");
    }
    HIPS(sv, e);
    sv->dev_allocs.push_back(p);
    return p;
}

size_t job_bytes(int mode, int Qp, int RP, int64_t N) {
    const size_t esz = mode == MODE_FP64 ? 8 : 4;
    return kAlign + 2 * align_up((size_t)Qp * N * esz) + 3 * align_up((size_t)RP * N * esz);
}

// Monitoring's share of a job's memory: U_r^T m (r x N), ||m_perp||^2 (N), the checks' sums.
size_t monitor_bytes(int r, int64_t N, int nchecks) {
    if (nchecks == 0) return 0;
    return align_up((size_t)r * N * 8) + align_up((size_t)N * 8) + align_up((size_t)nchecks * ST_COUNT * 8);
}

Consts &get_consts(ssmap_server *sv, Dict &d, const Job &j, int li) {
    uint64_t bb;
    std::memcpy(&bb, &j.st.beta, 8);
    auto key = std::make_tuple(j.mode, j.r, bb);
    auto it = d.consts.find(key);
    if (it != d.consts.end()) {
        fence_wait(sv, li, it->second.ready);
        return it->second;
    }
    HostConsts hc;
    host_consts(j.mode, d.U, d.s, d.V, d.kmin, d.P, d.Q, d.Qp, j.r, j.RP, j.st.beta, true, hc);
    Consts c;
    c.mode = j.mode;
    c.r = j.r;
    c.RP = j.RP;
    c.V = dev_alloc(sv, hc.V.size());
    c.b = dev_alloc(sv, hc.b.size());
    c.Vop = dev_alloc(sv, hc.Vop.size());
    c.Ur = (double *)dev_alloc(sv, hc.Ur.size() * 8);
    c.sig = (double *)dev_alloc(sv, hc.sig.size() * 8);
    c.acoef = (double *)dev_alloc(sv, hc.a.size() * 8);
    upload(sv, li, c.V, hc.V.data(), hc.V.size());
    upload(sv, li, c.b, hc.b.data(), hc.b.size());
    upload(sv, li, c.Vop, hc.Vop.data(), hc.Vop.size());
    upload(sv, li, c.Ur, hc.Ur.data(), hc.Ur.size() * 8);
    upload(sv, li, c.sig, hc.sig.data(), hc.sig.size() * 8);
    upload(sv, li, c.acoef, hc.a.data(), hc.a.size() * 8);
    c.ready.seq[li] = fence_record(sv, li);
    return d.consts.emplace(key, c).first->second;
}

// Size band of a job by the bytes one iteration moves: a job shares launches
// only with jobs of its band, so a small job's iteration is not as long as a
// large job's (< 64 MB, < 1 GB, larger).
int size_band(const ssmap_server *sv, const Job &j) {
    const double bytes = (double)j.g.N * (2.0 * sv->dicts[j.dict].Qp + 5.0 * j.RP) *
                         (j.mode == MODE_FP64 ? 8.0 : 4.0);
    return bytes < 64e6 ? 0 : bytes < 1e9 ? 1 : 2;
}

int find_class(ssmap_server *sv, const Job &j) {
    const FusedShape sh = default_shape(j.mode, j.g);
    const int rk = j.mode == MODE_BF16X3 ? j.RP : bucket_rank(j.r);
    const int band = size_band(sv, j);
    int in_band = 0;
    for (size_t c = 0; c < sv->classes.size(); ++c) {
        const Class &C = sv->classes[c];
        if (C.mode == j.mode && C.RP == j.RP && C.rkey == rk && C.shape.ty == sh.ty &&
            C.shape.tz == sh.tz && C.band == band)
            return (int)c;
        in_band += C.band == band;
    }
    Class C;
    C.mode = j.mode;
    C.RP = j.RP;
    C.rkey = rk;
    C.shape = sh;
    C.band = band;
    // small and middle bands get a stream each, the large band the rest, so
    // short launches never queue behind long ones in one stream
    const int L = sv->nlanes;
    if (band < 2) C.lane = std::min(band, L - 1);
    else C.lane = L > 2 ? 2 + in_band % (L - 2) : L - 1;
    sv->classes.push_back(C);
    sv->stats.classes = (int)sv->classes.size();
    return (int)sv->classes.size() - 1;
}

IterArgs args_at(const Job &j, int parity) {
    IterArgs a = j.a;
    a.z = j.z[parity];
    a.znew = j.z[parity ^ 1];
    return a;
}

// Rebuild a class's descriptor and brick tables from its members.
void upload_tables(ssmap_server *sv, Class &C) {
    std::vector<IterArgs> args(2 * C.members.size());
    std::vector<TileRef> tiles;
    std::vector<std::vector<TileRef>> per(C.members.size());
    size_t ntiles = 0;
    double bytes = 0;
    for (size_t k = 0; k < C.members.size(); ++k) {
        Job &j = sv->jobs[C.members[k]];
        args[2 * k] = args_at(j, 0);
        args[2 * k + 1] = args_at(j, 1);
        args[2 * k].phase = args[2 * k + 1].phase = (int)(j.r0 & 1);
        append_tiles(j.g, (int)k, C.mode, C.shape, per[k], j.code.empty() ? nullptr : &j.code);
        ntiles += per[k].size();
        const size_t esz = j.mode == MODE_FP64 ? 8 : 4;
        bytes += (double)j.g.N * (2.0 * j.a.nchunk * QC + 5.0 * j.RP) * esz;
    }
    // jobs with the most chunks first when workgroup b takes brick b (the brick
    // count not a multiple of 8), as for batches; a job's bricks stay contiguous
    std::vector<size_t> order(C.members.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    if (ntiles % 8 != 0)
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
            return args[2 * x].nchunk > args[2 * y].nchunk;
        });
    for (size_t k : order) {
        Job &j = sv->jobs[C.members[k]];
        j.tile_off = (int)tiles.size();
        tiles.insert(tiles.end(), per[k].begin(), per[k].end());
        j.tile_cnt = (int)per[k].size();
    }
    if (args.size() > C.cap_jobs) {
        C.cap_jobs = std::max<size_t>(2 * args.size(), 16);
        C.djobs = (IterArgs *)dev_alloc(sv, C.cap_jobs * sizeof(IterArgs));
    }
    if (tiles.size() > C.cap_tiles) {
        C.cap_tiles = std::max<size_t>(2 * tiles.size(), 1024);
        C.dtiles = (TileRef *)dev_alloc(sv, C.cap_tiles * sizeof(TileRef));
    }
    bool monitored = false;
    for (int64_t id : C.members) monitored |= sv->jobs[id].check_every > 0;
    if (monitored && tiles.size() > C.cap_mon) {
        C.cap_mon = std::max<size_t>(2 * tiles.size(), 1024);
        C.dmon = (double *)dev_alloc(sv, C.cap_mon * sizeof(double));
    }
    upload(sv, C.lane, C.djobs, args.data(), args.size() * sizeof(IterArgs));
    upload(sv, C.lane, C.dtiles, tiles.data(), tiles.size() * sizeof(TileRef));
    C.ntiles = (int)tiles.size();
    C.maxchunk = 0;
    for (const IterArgs &a : args) C.maxchunk = std::max(C.maxchunk, a.nchunk);
    C.model_ms = kLaunchMs + bytes / kBytesPerMs;
    C.dirty = false;
}

// A job starts iterating: it joins its class at the class's current round.
void start_job(ssmap_server *sv, int64_t id) {
    Job &j = sv->jobs[id];
    Class &C = sv->classes[j.cls];
    j.r0 = C.round;
    C.members.push_back(id);
    C.dirty = true;
}

// The next waiting large job, if none is running.
void start_next_large(ssmap_server *sv) {
    if (sv->large_running >= 0 || sv->large_wait.empty()) return;
    sv->large_running = sv->large_wait.front();
    sv->large_wait.pop_front();
    start_job(sv, sv->large_running);
}

// Output, flag read-back, completion event and release of the job's memory.
void retire(ssmap_server *sv, Job &j, int li) {
    hipStream_t s = sv->lanes[li].s;
    launch_output(j.mode, j.z[j.iters & 1], j.dF, sv->dicts[j.dict].Q, j.g.N, false, s);
    HIPS(sv, hipGetLastError());
    HIPS(sv, hipMemcpyAsync(&sv->flags[j.slot], j.bad, sizeof(int), hipMemcpyDeviceToHost, s));
    if (!j.hist_iter.empty())
        HIPS(sv, hipMemcpyAsync(sv->hist_pinned + (size_t)j.slot * kServedChecks * ST_COUNT, j.hist,
                                j.hist_iter.size() * ST_COUNT * 8, hipMemcpyDeviceToHost, s));
    j.done_ev = get_event(sv, true);
    HIPS(sv, hipEventRecord(j.done_ev, s));
    Fence f;
    f.seq[li] = fence_record(sv, li);
    sv->slab.release(j.off, j.bytes, f);
    j.retired = true;
}

// Admit the head of the queue if its state fits; false otherwise.
bool admit_one(ssmap_server *sv) {
    if (sv->queue.empty() || sv->free_slots.empty()) return false;
    const int64_t id = sv->queue.front();
    Job &j = sv->jobs[id];
    size_t off = 0;
    Fence f;
    if (!sv->slab.alloc(j.bytes, off, f)) return false;
    sv->queue.pop_front();
    j.off = off;
    j.slot = sv->free_slots.back();
    sv->free_slots.pop_back();
    j.cls = find_class(sv, j);
    Class &C = sv->classes[j.cls];
    const int li = C.lane;
    hipStream_t s = sv->lanes[li].s;
    fence_wait(sv, li, f);
    Dict &d = sv->dicts[j.dict];
    Consts &cs = get_consts(sv, d, j, li);

    const int64_t N = j.g.N;
    const size_t esz = j.mode == MODE_FP64 ? 8 : 4;
    const size_t zb = align_up((size_t)d.Qp * N * esz), rb = align_up((size_t)j.RP * N * esz);
    uint8_t *p = sv->slab_base + off;
    j.bad = (int *)p;
    p += kAlign;
    j.z[0] = p;
    j.z[1] = p + zb;
    void *w = p + 2 * zb, *y = p + 2 * zb + rb, *ah = p + 2 * zb + 2 * rb;
    if (!j.code.empty()) {
        j.dcode = p + 2 * zb + 3 * rb + monitor_bytes(j.r, N, j.nchecks);
        upload(sv, li, j.dcode, j.code.data(), j.code.size());
    }
    if (j.check_every > 0) {
        uint8_t *mp = p + 2 * zb + 3 * rb;
        j.t = (double *)mp;
        j.mperp2 = (double *)(mp + align_up((size_t)j.r * N * 8));
        j.hist = (double *)(mp + align_up((size_t)j.r * N * 8) + align_up((size_t)N * 8));
        j.sig = cs.sig;
        if (!sv->hist_pinned)
            HIPS(sv, hipHostMalloc((void **)&sv->hist_pinned,
                                   (size_t)kFlagSlots * kServedChecks * ST_COUNT * sizeof(double)));
        if (!sv->lane_partial[li])
            sv->lane_partial[li] = (double *)dev_alloc(sv, (size_t)kMonitorBlocks * ST_COUNT * 8);
    }

    IterArgs &a = j.a;
    a = IterArgs{};
    a.w = w;
    a.y = y;
    a.ah = ah;
    a.V = cs.V;
    a.bcoef = cs.b;
    a.Vu = cs.Vop;
    a.r = j.r;
    a.RP = j.RP;
    a.nchunk = d.nchunk;
    a.g = j.g;
    a.tau = j.tau;
    a.lam2 = 2.0 * j.lambda;
    a.beta = j.st.beta;
    a.code = j.dcode;

    // a1: projection and z^0 = 0, w^0 = a.h, y^0 = 0
    launch_zero(j.bad, 1, 4, s);
    launch_project(j.mode, j.dM, d.P, cs.Ur, cs.sig, cs.acoef, j.r, j.RP, N, j.t, j.mperp2, ah,
                   w, y, j.bad, j.dcode, s);
    launch_zero(j.z[0], (size_t)d.Qp * N, (int)esz, s);
    launch_zero(j.z[1], (size_t)d.Qp * N, (int)esz, s);
    HIPS(sv, hipGetLastError());
    j.state = RUNNING;
    j.admit_ms = host_ms(sv);
    sv->stats.admitted++;
    if (j.iters == 0) {
        retire(sv, j, li);
        return true;
    }
    if (C.band == 2) {
        sv->large_wait.push_back(id);
        start_next_large(sv);
    } else {
        start_job(sv, id);
    }
    return true;
}

void reap(ssmap_server *sv, Job &j) {
    if (j.state != RUNNING || !j.retired || !event_done(sv, j.done_ev)) return;
    float ms = 0.0f;
    HIPS(sv, hipEventElapsedTime(&ms, sv->epoch, j.done_ev));
    j.done_ms = (double)ms;
    put_event(sv, j.done_ev, true);
    j.done_ev = nullptr;
    j.status = sv->flags[j.slot] ? SSMAP_ENONFINITE : SSMAP_OK;
    if (!j.hist_iter.empty()) {
        const double *h = sv->hist_pinned + (size_t)j.slot * kServedChecks * ST_COUNT;
        j.hist_sums.assign(h, h + j.hist_iter.size() * ST_COUNT);
        for (size_t i = 0; i < j.hist_iter.size(); ++i)
            if (h[i * ST_COUNT + ST_NONFINITE] != 0.0 || !std::isfinite(h[i * ST_COUNT + ST_DATA]))
                j.status = SSMAP_ENONFINITE;
    }
    sv->free_slots.push_back(j.slot);
    j.slot = -1;
    j.state = DONE;
    sv->stats.completed++;
    sv->stats.voxel_iterations += (double)j.g.N * j.iters;
}

void reap_all(ssmap_server *sv) {
    for (auto &j : sv->jobs) reap(sv, j);
    for (int li = 0; li < sv->nlanes; ++li) lane_poll(sv, li);
}

int pending(const ssmap_server *sv) {
    int n = 0;
    for (const auto &j : sv->jobs) n += j.state != DONE;
    return n;
}

// Fold a finished chunk's measured round time into the class's estimate.
void close_chunk(ssmap_server *sv, Class &C) {
    Class::Chunk ch = C.chunks.front();
    C.chunks.pop_front();
    HIPS(sv, hipEventSynchronize(ch.end));
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ch.start, ch.end) == hipSuccess && ch.rounds > 0 && C.model_ms > 0) {
        const double r = std::clamp((double)ms / ch.rounds / C.model_ms, 0.25, 64.0);
        C.ratio = 0.5 * C.ratio + 0.5 * r;
    }
    put_event(sv, ch.start, true);
    put_event(sv, ch.end, true);
}

// Whether a monitored job takes a check once its class has run `round` rounds
// (every check_every-th iteration of the job and its last).
bool checked_after_round(const Job &j, int64_t round) {
    if (j.check_every <= 0) return false;
    const int64_t done = round - j.r0;
    return done > 0 && done <= j.iters && (done % j.check_every == 0 || done == j.iters);
}

// The reductions of a job's check after its iteration `done` (z^done against
// z^{done-1}, y^done from the job's r-vector state, the per-brick sums of the
// class's monitored launch), in stream order, into the job's next check slot.
void monitor_job(ssmap_server *sv, const Class &C, Job &j, hipStream_t s) {
    const Dict &d = sv->dicts[j.dict];
    const int done = (int)(C.round - j.r0);
    if ((int)j.hist_iter.size() >= j.nchecks) sfail(SSMAP_EINVAL, "more monitor checks than planned");
    MonArgs m{};
    m.z = j.z[done & 1];
    m.y = j.a.y;
    m.dzpart = C.dmon + j.tile_off;
    m.ndz = j.tile_cnt;
    m.sig = j.sig;
    m.t = j.t;
    m.mperp2 = j.mperp2;
    m.r = j.r;
    m.RP = j.RP;
    m.Q = d.Q;
    m.g = j.g;
    m.nchunk = d.nchunk;
    m.code = j.dcode;
    launch_monitor(j.mode, m, sv->lane_partial[C.lane], j.hist + j.hist_iter.size() * ST_COUNT, s);
    HIPS(sv, hipGetLastError());
    j.hist_iter.push_back(done);
}

// Enqueue about horizon_ms of rounds for class C (at most two chunks per
// class in flight: the host waits for the older one first).
void run_class(ssmap_server *sv, Class &C, double horizon_ms) {
    if (C.members.empty()) return;
    if (C.chunks.size() >= 2) close_chunk(sv, C);
    hipStream_t s = sv->lanes[C.lane].s;
    if (C.dirty) upload_tables(sv, C);
    const double est = std::max(1e-3, C.model_ms * C.ratio);
    const int64_t rounds =
        std::max<int64_t>(1, std::min<int64_t>(4096, (int64_t)std::ceil(horizon_ms / est)));
    Class::Chunk ch{get_event(sv, true), get_event(sv, true), 0};
    HIPS(sv, hipEventRecord(ch.start, s));
    for (int64_t i = 0; i < rounds && !C.members.empty(); ++i) {
        if (C.dirty) upload_tables(sv, C);
        FusedLaunch L{};
        L.mode = C.mode;
        L.r = C.rkey;
        L.RP = C.RP;
        L.shape = C.shape;
        L.jobs = C.djobs;
        L.tiles = C.dtiles;
        L.ntiles = C.ntiles;
        L.maxchunk = C.maxchunk;
        L.round = (int)(C.round & 0x3fffffff);   // only the parity matters
        // member jobs whose check falls after this round: the monitored build sums
        // (z^{k+1} - z^k)^2 per brick, then each such job's reductions follow
        bool any_check = false;
        for (int64_t id : C.members) any_check |= checked_after_round(sv->jobs[id], C.round + 1);
        L.mon = any_check ? C.dmon : nullptr;
        if (!launch_fused(L, s)) sfail(SSMAP_EINVAL, "no fused kernel for this class");
        sv->stats.launches++;
        ch.rounds++;
        C.round++;
        if (any_check)
            for (int64_t id : C.members)
                if (checked_after_round(sv->jobs[id], C.round)) monitor_job(sv, C, sv->jobs[id], s);
        for (size_t k = 0; k < C.members.size();) {
            Job &j = sv->jobs[C.members[k]];
            if (C.round - j.r0 == j.iters) {
                const int64_t id = C.members[k];
                retire(sv, j, C.lane);
                C.members.erase(C.members.begin() + (ptrdiff_t)k);
                C.dirty = true;
                if (id == sv->large_running) {
                    sv->large_running = -1;
                    start_next_large(sv);    // may join this class at once
                }
            } else {
                ++k;
            }
        }
    }
    HIPS(sv, hipGetLastError());
    HIPS(sv, hipEventRecord(ch.end, s));
    C.chunks.push_back(ch);
}

void pump_impl(ssmap_server *sv, double horizon_ms) {
    reap_all(sv);
    while (admit_one(sv)) {
    }
    bool any = false;
    for (auto &C : sv->classes) {
        any |= !C.members.empty();
        run_class(sv, C, horizon_ms);
    }
    if (!any) {                          // nothing to iterate: let retirements finish
        for (int li = 0; li < sv->nlanes; ++li) HIPS(sv, hipStreamSynchronize(sv->lanes[li].s));
    }
    reap_all(sv);
    sv->stats.in_use_bytes = (double)sv->slab.used();
    sv->stats.peak_bytes = (double)sv->slab.peak();
}

template <typename Fn>
ssmap_status sv_guarded(ssmap_server *sv, Fn &&fn) {
    try {
        if (sv && sv->poisoned) sfail(SSMAP_EDEVICE, "server poisoned by an earlier device error");
        fn();
        return SSMAP_OK;
    } catch (const SvFail &f) {
        if (sv) sv->err = f.msg;
        else g_server_create_error = f.msg;
        return f.status;
    } catch (const std::bad_alloc &) {
        if (sv) sv->err = "host allocation failed";
        else g_server_create_error = "host allocation failed";
        return SSMAP_ENOMEM;
    } catch (...) {
        if (sv) {
            sv->err = "unexpected internal error";
            sv->poisoned = true;
        } else {
            g_server_create_error = "unexpected internal error";
        }
        return SSMAP_EDEVICE;
    }
}

void free_server(ssmap_server *sv) {
    if (!sv) return;
    for (int li = 0; li < sv->nlanes; ++li)
        if (sv->lanes[li].s) (void)hipStreamSynchronize(sv->lanes[li].s);
    for (auto &L : sv->lanes) {
        for (auto &pe : L.pend) (void)hipEventDestroy(pe.second);
        if (L.s) (void)hipStreamDestroy(L.s);
    }
    for (auto &r : sv->stage_live) (void)hipEventDestroy(r.ev);
    for (auto &C : sv->classes)
        for (auto &ch : C.chunks) {
            (void)hipEventDestroy(ch.start);
            (void)hipEventDestroy(ch.end);
        }
    for (auto &j : sv->jobs)
        if (j.done_ev) (void)hipEventDestroy(j.done_ev);
    for (hipEvent_t e : sv->fence_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : sv->timing_pool) (void)hipEventDestroy(e);
    if (sv->epoch) (void)hipEventDestroy(sv->epoch);
    for (void *p : sv->dev_allocs) (void)hipFree(p);
    if (sv->slab_base) (void)hipFree(sv->slab_base);
    if (sv->stage) (void)hipHostFree(sv->stage);
    if (sv->flags) (void)hipHostFree(sv->flags);
    if (sv->hist_pinned) (void)hipHostFree(sv->hist_pinned);
    delete sv;
}

}  // namespace

extern "C" {

ssmap_status ssmap_server_create(const ssmap_server_opts *opts, ssmap_server **out) {
    if (out) *out = nullptr;
    ssmap_server *sv = nullptr;
    ssmap_status st = sv_guarded(nullptr, [&] {
        if (!opts || !out) sfail(SSMAP_EINVAL, "NULL argument");
        if (!(std::isfinite(opts->hbm_budget) && opts->hbm_budget >= (double)kAlign))
            sfail(SSMAP_EINVAL, "hbm_budget must be a finite byte count >= 256");
        if (opts->streams < 0 || opts->streams > kMaxLanes)
            sfail(SSMAP_EINVAL, "streams must be in [0, 4]");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
            (void)hipGetLastError();
            sfail(SSMAP_ENODEV, "no HIP device");
        }
        sv = new ssmap_server();
        if (hipGetDevice(&sv->device) != hipSuccess) sfail(SSMAP_ENODEV, "hipGetDevice failed");
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, sv->device) != hipSuccess)
            sfail(SSMAP_ENODEV, "hipGetDeviceProperties failed");
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            sfail(SSMAP_ENODEV, std::string("device is ") + prop.gcnArchName + ", need gfx950");
        const size_t budget = (size_t)opts->hbm_budget / kAlign * kAlign;
        const hipError_t e = hipMalloc((void **)&sv->slab_base, budget);
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            sfail(SSMAP_ENOMEM, "cannot reserve the device-memory budget");
        }
        HIPS(sv, e);
        sv->budget = (double)budget;
        sv->slab.init(budget);
        sv->nlanes = opts->streams == 0 ? kMaxLanes : opts->streams;
        for (int li = 0; li < sv->nlanes; ++li)
            HIPS(sv, hipStreamCreateWithFlags(&sv->lanes[li].s, hipStreamNonBlocking));
        HIPS(sv, hipHostMalloc((void **)&sv->stage, kStagingBytes));
        HIPS(sv, hipHostMalloc((void **)&sv->flags, kFlagSlots * sizeof(int)));
        for (int i = kFlagSlots - 1; i >= 0; --i) sv->free_slots.push_back(i);
        HIPS(sv, hipEventCreate(&sv->epoch));
        HIPS(sv, hipEventRecord(sv->epoch, sv->lanes[0].s));
        HIPS(sv, hipEventSynchronize(sv->epoch));
        sv->t0 = Clock::now();
        sv->stats.budget_bytes = sv->budget;
        sv->stats.streams = sv->nlanes;
        *out = sv;
    });
    if (st != SSMAP_OK) {
        free_server(sv);
        if (out) *out = nullptr;
    }
    return st;
}

ssmap_status ssmap_server_add_dictionary(ssmap_server *sv, const double *K, int P, int Q,
                                         int *dict_id) {
    if (!sv) return SSMAP_EINVAL;
    return sv_guarded(sv, [&] {
        if (!K || !dict_id) sfail(SSMAP_EINVAL, "NULL argument");
        if (P < 1 || Q < 1) sfail(SSMAP_EINVAL, "P and Q must be >= 1");
        double fro = 0.0;
        for (size_t i = 0; i < (size_t)P * Q; ++i) {
            if (!std::isfinite(K[i])) sfail(SSMAP_ENONFINITE, "K holds a NaN or Inf");
            fro += K[i] * K[i];
        }
        if (!(fro > 0)) sfail(SSMAP_EINVAL, "K is zero");
        Dict d;
        d.P = P;
        d.Q = Q;
        d.kmin = std::min(P, Q);
        d.Qp = (Q + QC - 1) / QC * QC;
        d.nchunk = d.Qp / QC;
        thin_svd(K, P, Q, d.U, d.s, d.V);
        sv->dicts.push_back(std::move(d));
        *dict_id = (int)sv->dicts.size() - 1;
    });
}

ssmap_status ssmap_server_submit_masked(ssmap_server *sv, int dict_id, const int64_t grid[3],
                                        const uint8_t *mask, const void *dM, double lambda,
                                        const ssmap_steps *steps, int iters, void *dF, int64_t *job_id) {
    if (!sv) return SSMAP_EINVAL;
    return sv_guarded(sv, [&] {
        if (!grid || !dM || !dF || !steps || !job_id) sfail(SSMAP_EINVAL, "NULL argument");
        if (dict_id < 0 || dict_id >= (int)sv->dicts.size()) sfail(SSMAP_EINVAL, "unknown dictionary");
        const Dict &d = sv->dicts[dict_id];
        for (int i = 0; i < 3; ++i)
            if (grid[i] < 1) sfail(SSMAP_EINVAL, "grid dimensions must be >= 1");
        const double Nd = (double)grid[0] * (double)grid[1] * (double)grid[2];
        if (Nd * d.Qp > 9.0e18) sfail(SSMAP_EINVAL, "grid too large");
        const ssmap_steps &st = *steps;
        if (!(std::isfinite(lambda) && lambda >= 0)) sfail(SSMAP_EINVAL, "lambda must be finite and >= 0");
        if (!(std::isfinite(st.beta) && st.beta > 0)) sfail(SSMAP_EINVAL, "beta must be finite and > 0");
        if (!std::isfinite(st.xi_p)) sfail(SSMAP_EINVAL, "xi_p must be finite");
        if (iters < 0) sfail(SSMAP_EINVAL, "iters must be >= 0");
        if (st.rank < -1 || st.rank > d.kmin) sfail(SSMAP_EINVAL, "rank must be in [-1, min(P,Q)]");
        if (st.precision < SSMAP_FP64 || st.precision > SSMAP_BF16X3)
            sfail(SSMAP_EINVAL, "unknown precision");
        if (st.check_every < 0 || st.flags != 0 || st.stop_tol != 0)
            sfail(SSMAP_EINVAL, "served jobs take no flags and no stopping rule; check_every >= 0");
        const int nchecks = st.check_every > 0 && iters > 0
                                ? iters / st.check_every + (iters % st.check_every != 0) : 0;
        if (nchecks > kServedChecks)
            sfail(SSMAP_EINVAL, "a served job takes at most " + std::to_string(kServedChecks) +
                                    " monitor checks (iters / check_every)");
        if (st.kernel != SSMAP_KERNEL_AUTO && st.kernel != SSMAP_KERNEL_FUSED)
            sfail(SSMAP_EINVAL, "served jobs run the fused kernel");
        Job j;
        j.dict = dict_id;
        j.g = Grid{grid[0], grid[1], grid[2], grid[0] * grid[1] * grid[2]};
        j.dM = dM;
        j.dF = dF;
        j.lambda = lambda;
        j.st = st;
        j.iters = iters;
        j.mode = st.precision;
        j.r = rank_rule(d.s, st.rank);
        j.RP = (j.r + 15) / 16 * 16;
        if (!fused_supported(j.mode, j.RP, j.g.N))
            sfail(SSMAP_EINVAL, "no fused kernel for this precision, rank and size");
        double dtd = 0.0;
        if (mask) {                      // the graph the mask induces (as ssmap_set_mask)
            int64_t inside = 0;
            mask_codes(j.g, mask, j.code, inside);
            dtd = masked_dtd_norm(j.g, j.code);
        } else {
            dtd = dtd_norm_closed(j.g);
        }
        j.dtd = dtd;
        j.xi = st.xi_p > 0 ? st.xi_p : kXiFactor * lambda * dtd + kEpsXi;
        j.tau = 1.0 / (j.xi + st.beta);
        j.check_every = nchecks > 0 ? st.check_every : 0;
        j.nchecks = nchecks;
        j.bytes = job_bytes(j.mode, d.Qp, j.RP, j.g.N) + monitor_bytes(j.r, j.g.N, nchecks) +
                  (mask ? align_up((size_t)j.g.N) : 0);
        if ((double)j.bytes > sv->budget)
            sfail(SSMAP_ENOMEM, "job needs " + std::to_string(j.bytes) +
                                    " device bytes, above the server budget");
        j.submit_ms = host_ms(sv);
        sv->jobs.push_back(j);
        *job_id = (int64_t)sv->jobs.size() - 1;
        sv->queue.push_back(*job_id);
        sv->stats.submitted++;
    });
}

ssmap_status ssmap_server_submit(ssmap_server *sv, int dict_id, const int64_t grid[3],
                                 const void *dM, double lambda, const ssmap_steps *steps,
                                 int iters, void *dF, int64_t *job_id) {
    return ssmap_server_submit_masked(sv, dict_id, grid, nullptr, dM, lambda, steps, iters, dF, job_id);
}

ssmap_status ssmap_server_pump(ssmap_server *sv, double horizon_ms, int *n_pending) {
    if (!sv) return SSMAP_EINVAL;
    return sv_guarded(sv, [&] {
        if (!(std::isfinite(horizon_ms) && horizon_ms > 0)) sfail(SSMAP_EINVAL, "horizon_ms must be > 0");
        pump_impl(sv, horizon_ms);
        if (n_pending) *n_pending = pending(sv);
    });
}

ssmap_status ssmap_server_poll(ssmap_server *sv, int64_t job_id, ssmap_job_info *out) {
    if (!sv) return SSMAP_EINVAL;
    return sv_guarded(sv, [&] {
        if (!out) sfail(SSMAP_EINVAL, "NULL argument");
        if (job_id < 0 || job_id >= (int64_t)sv->jobs.size()) sfail(SSMAP_EINVAL, "unknown job");
        Job &j = sv->jobs[job_id];
        reap(sv, j);
        std::memset(out, 0, sizeof(*out));
        out->state = j.state;
        out->status = j.status;
        out->rank = j.r;
        out->rank_padded = j.RP;
        out->precision = j.mode;
        out->iters = j.iters;
        out->xi_p = j.xi;
        out->state_bytes = (double)j.bytes;
        out->submit_ms = j.submit_ms;
        out->admit_ms = j.admit_ms;
        out->done_ms = j.done_ms;
    });
}

ssmap_status ssmap_server_get_job_stats(ssmap_server *sv, int64_t job_id, ssmap_stats *out) {
    if (!sv) return SSMAP_EINVAL;
    return sv_guarded(sv, [&] {
        if (!out) sfail(SSMAP_EINVAL, "NULL argument");
        if (job_id < 0 || job_id >= (int64_t)sv->jobs.size()) sfail(SSMAP_EINVAL, "unknown job");
        Job &j = sv->jobs[job_id];
        reap(sv, j);
        if (j.state != DONE) sfail(SSMAP_EINVAL, "job " + std::to_string(job_id) + " is not done");
        std::memset(out, 0, sizeof(*out));
        out->rank = j.r;
        out->rank_padded = j.RP;
        out->precision = j.mode;
        out->kernel = SSMAP_KERNEL_FUSED;
        out->iters = j.iters;
        out->xi_p = j.xi;
        out->tau = j.tau;
        out->dtd_norm = j.dtd;
        out->sigma_max = sv->dicts[j.dict].s.empty() ? 0.0 : sv->dicts[j.dict].s[0];
        out->device_bytes = (double)j.bytes;
        // the checks' sums as the single solve records them (Eq. spat, the dual residual, ||z||)
        const int n = (int)std::min<size_t>(j.hist_iter.size(), SSMAP_MAX_HIST);
        for (int i = 0; i < n; ++i) {
            const double *h = j.hist_sums.data() + (size_t)i * ST_COUNT;
            out->hist_iter[i] = j.hist_iter[i];
            out->hist_objective[i] = 0.5 * h[ST_DATA] + j.lambda * h[ST_REG];
            out->hist_dual[i] = j.st.beta * std::sqrt(h[ST_DZ]);
            out->hist_znorm[i] = std::sqrt(h[ST_ZNORM]);
            out->hist_primal[i] = -1.0;
            out->hist_dfcs[i] = -1.0;
            out->hist_dfcs_f[i] = -1.0;
        }
        out->n_hist = n;
    });
}

ssmap_status ssmap_server_drain(ssmap_server *sv) {
    if (!sv) return SSMAP_EINVAL;
    return sv_guarded(sv, [&] {
        while (pending(sv) > 0) pump_impl(sv, 20.0);
        for (int li = 0; li < sv->nlanes; ++li) HIPS(sv, hipStreamSynchronize(sv->lanes[li].s));
        reap_all(sv);
    });
}

ssmap_status ssmap_server_get_stats(const ssmap_server *sv, ssmap_server_stats *out) {
    if (!sv || !out) return SSMAP_EINVAL;
    *out = sv->stats;
    return SSMAP_OK;
}

const char *ssmap_server_last_error(const ssmap_server *sv) {
    return sv ? sv->err.c_str() : g_server_create_error.c_str();
}

void ssmap_server_destroy(ssmap_server *sv) { free_server(sv); }

}  // extern "C"
