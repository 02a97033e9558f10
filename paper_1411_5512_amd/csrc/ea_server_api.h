// ea_server_api.h -- the serving form (ea_server_* in ea.h): continuous
// batching of a stream of simulation jobs.
//
// Jobs are admitted first-come first-served while their device footprint
// fits a fixed HBM budget (a first-fit pool carved from one allocation) and
// a slot is free.  Admitted jobs keep their lattices resident in HBM; every
// epoch is one persistent launch that advances each resident job by a span of
// sweeps sized so that all units take about the same time (a fixed number of
// site-sweeps per replica), taking the job's scheduled snapshots and
// measurements on the way.  Between epochs finished jobs hand their results
// to the host and free their memory, and waiting jobs are admitted.  Epochs
// run on the calling thread (ea_server_step) or on a worker thread
// (ea_server_start), so that requests that arrive while a launch is on the
// GPU join at the next epoch.  Results are the same integers as a run alone:
// the dynamics never depend on how the sweeps are split or what else runs.
//
// Lattices too large for one workgroup's LDS (L > 64) are "streamed" jobs:
// each is a plain-form simulation placed in its pool region, advanced in the
// epoch by slab launches (ea_set_slab_plan) from up to kStreamWorkers
// worker threads at once, beside the epoch's batched launch on the compute units it
// leaves free (each epoch's slab plans are sized to them), or after it when
// it leaves fewer than a quarter (persistent slab workgroups beside a
// batched launch that fills the device would wait for its compute units
// while holding their own).  Each worker owns one stream, and a streamed job runs
// on the stream of the worker it was given at admission (the one with the
// least remaining work): streams share the process's hardware queues in
// turn, and two persistent launches on one queue run one after the other,
// so the workers are as many as the queues left beside the batched stream's
// (GPU_MAX_HW_QUEUES, 4 by default) allow.  A streamed job's span is sized
// by time (its own measured seconds per sweep), so that the streamed work of
// an epoch takes about as long as the previous epoch's batched launch.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace {

using steady = std::chrono::steady_clock;

constexpr int kStreamWorkers = 4;  // at most this many host threads drive streamed jobs

// Workers that can run their persistent launches at the same time: the
// process's hardware queues (HIP's GPU_MAX_HW_QUEUES, 4 unless set) less the
// one the batched stream takes, at least 1 and at most kStreamWorkers.
int server_stream_workers()
{
    int queues = 4;
    if (const char *e = std::getenv("GPU_MAX_HW_QUEUES")) {
        const int v = std::atoi(e);
        if (v > 0) queues = v;
    }
    return std::max(1, std::min(kStreamWorkers, queues - 1));
}

// First-fit allocator over one device buffer (offsets, 256-byte granules).
struct DevicePool {
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    size_t in_use = 0, peak = 0;

    void reset(size_t n)
    {
        size = n;
        free_.clear();
        if (n) free_[0] = n;
        in_use = peak = 0;
    }
    bool alloc(size_t n, size_t *off)
    {
        n = align256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                in_use += n;
                peak = std::max(peak, in_use);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = align256(n);
        in_use -= n;
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum { SJ_PENDING = 0, SJ_RUNNING = 1, SJ_DONE = 2 };

struct ServerJob {
    uint64_t id = 0;
    BatchJobHost h;
    size_t pool_off = 0;
    steady::time_point t_submit, t_done;
    std::vector<unsigned long long> results;  // [n_meas][obs_stride] after completion
    bool streamed = false;                     // on the slab path (L > 64, or given it), on a worker's stream
    int worker = 0;                            // that worker (its stream)
    int plan_K = 0;                            // its slab plan's slabs per replica (-1: half-step launches)
    ea_sim *sim = nullptr;                     // its simulation, in the pool region
    int next_meas = 0, next_tw = 0;            // schedule positions of a streamed job
    double sweep_s = 0.0;                      // measured seconds per sweep of a streamed job
};

ea_status plan_server_job(const ea_job &in, ServerJob &j)
{
    if (!valid_L(in.L)) return fail(EA_ERR_ARG, "L=%d must be a multiple of 8 in [8, %d]", in.L, kMaxL);
    j.streamed = !batch_L_ok(in.L);
    return j.streamed ? plan_streamed_job(in, 0, j.h) : plan_job(in, 0, j.h);
}

}  // namespace

struct ea_server {
    ea_server_opts opts{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<hipStream_t> wstreams;  // one per streamed-job worker
    int n_cu = 0;                       // compute units of the device
    hipEvent_t ev_batch[2] = {nullptr, nullptr};  // around each batched launch
    double last_batch_s = 0.0;                    // duration of the last batched launch
    char *pool_buf = nullptr;
    DevicePool pool;
    ea::BatchJobDev *d_jobs = nullptr;
    ea::BatchUnit *d_units = nullptr;
    size_t lds_bytes = 0;

    std::mutex mu;  // guards everything below
    std::condition_variable cv;
    std::deque<std::unique_ptr<ServerJob>> pending;
    std::vector<std::unique_ptr<ServerJob>> resident;
    std::unordered_map<uint64_t, std::unique_ptr<ServerJob>> done;
    std::unordered_map<uint64_t, int> state_of;
    uint64_t next_id = 1, submitted = 0, admitted = 0, completed = 0, epochs = 0, streamed_small = 0, moved = 0;
    std::vector<double> latencies;
    double flips = 0.0, busy_s = 0.0;
    bool have_first = false;
    steady::time_point first_submit;

    std::thread worker;
    bool worker_on = false, stop = false;
    std::mutex epoch_mu;  // one epoch at a time
    std::string worker_error;
};

namespace {

// Advance a streamed job to t_stop on the second stream, taking the snapshots
// and measurements scheduled up to t_stop that it has not taken yet (those at
// t = 0 included); each measurement's integers become the job's result row in
// the batched kernel's counter form, so results are read back the same way.
ea_status server_advance_streamed(ServerJob &j, uint64_t t_stop)
{
    BatchJobHost &h = j.h;
    const int n_meas = h.job.n_meas, n_tw = h.job.n_tw;
    const int64_t N = (int64_t)h.job.L * h.job.L * h.job.L;
    std::vector<uint64_t> tw((size_t)n_tw);
    std::vector<int64_t> autocorr(2 * (size_t)n_tw), c4(3 * (size_t)(h.R + 1));
    uint64_t t = h.t_host;
    for (;;) {
        uint64_t te = ~0ull;
        if (j.next_tw < n_tw) te = std::min<uint64_t>(te, h.tw[(size_t)j.next_tw]);
        if (j.next_meas < n_meas) te = std::min<uint64_t>(te, h.meas_t[(size_t)j.next_meas]);
        if (te > t_stop) break;
        if (te > t) {
            ea_status st = ea_sweep(j.sim, te - t);
            if (st != EA_OK) return st;
            t = te;
        }
        if (j.next_tw < n_tw && h.tw[(size_t)j.next_tw] == te) {
            ea_status st = ea_snapshot(j.sim, j.next_tw);
            if (st != EA_OK) return st;
            ++j.next_tw;
        }
        if (j.next_meas < n_meas && h.meas_t[(size_t)j.next_meas] == te) {
            ea_obs o{};
            o.n_tw = n_tw;
            o.tw = tw.data();
            o.autocorr = autocorr.data();
            o.rmax = h.R;
            o.c4 = c4.data();
            ea_status st = ea_measure(j.sim, &o);
            if (st != EA_OK) return st;
            unsigned long long *m = j.results.data() + (size_t)j.next_meas * (size_t)h.obs_stride;
            for (int r = 0; r < 2; ++r) {
                m[ea::M_UNSAT + r] = (unsigned long long)o.unsat[r];
                m[ea::M_DOWN + r] = (unsigned long long)((N - o.mag[r]) / 2);
                for (int k = 0; k < n_tw; ++k)
                    m[ea::M_AUTO + 2 * k + r] = (unsigned long long)((N - o.autocorr[r * n_tw + k]) / 2);
            }
            m[ea::M_QDIFF] = (unsigned long long)((N - o.overlap) / 2);
            for (int i = 0; i < 3 * (h.R + 1); ++i)
                m[ea::M_AUTO + 2 * n_tw + i] = (unsigned long long)((N - o.c4[i]) / 2);
            ++j.next_meas;
        }
    }
    if (t_stop > t) return ea_sweep(j.sim, t_stop - t);
    return EA_OK;
}

// Streamed jobs run as slab launches (ea_set_slab_plan) from the workers'
// threads at once: each job's plan uses at most `share` compute units (two
// workgroups of one CU per slab), so that the slab launches in flight fit
// the CUs they are given together; a lattice whose slabs would not fit LDS
// at that share uses one launch per half-step (no co-residency needed).
void server_slab_plan(ServerJob &j, int share)
{
    const int K = std::min(std::max(1, share / 2), j.h.job.L);
    if (K == j.plan_K) return;
    if (ea_set_slab_plan(j.sim, K, 0) == EA_OK) {
        j.plan_K = K;
    } else if (j.plan_K != -1) {
        (void)ea_set_slab_plan(j.sim, -1, 0);
        j.plan_K = -1;
    }
}

// An LDS-sized job (L >= kLoneStreamL) admitted while some worker has no
// streamed job runs as a streamed job instead: alone in the batched kernel
// its two replicas would hold two CUs for the whole run while the rest of
// the device idles (an L = 64 job: 24.8 us per sweep there, about 2.3 us as
// a slab job on many CUs).  Re-plans j.h for the plain form's layout and
// returns true if it did.  Results never depend on the form.
constexpr int kLoneStreamL = 48;

bool stream_small_job(const ea_server *s, ServerJob &j)
{
    if (j.streamed || j.h.job.L < kLoneStreamL) return false;
    size_t n_streamed = 0;
    for (const auto &r : s->resident) n_streamed += r->streamed ? 1 : 0;
    if (n_streamed >= s->wstreams.size()) return false;
    const Layout lay = make_layout(j.h.job.L, j.h.job.n_tw, plain_rw(j.h.job.L));
    j.streamed = true;
    j.h.RW = lay.RW;
    j.h.W = lay.W;
    j.h.POS = j.h.job.L * j.h.job.L * lay.RW;
    j.h.bytes = align256(lay.total);
    return true;
}

// A batched job with at least this many site-sweeps left (about 50 ms of an
// L = 64 job in the batched kernel) may move to the slab path.
constexpr double kMoveMinSiteSweeps = 64.0 * 64 * 64 * 2000;

// Move batched job j to the slab path mid-run, on worker `worker`'s stream
// (a batched job that outlasts the rest would hold two CUs while the device
// idles).  The plain run is rebuilt through the ABI from the job's packed
// state: its snapshots taken so far, each restored at its time, then the
// current spins and time; the couplings are regenerated from the same keys.
// The measurements taken so far go to the host as the job's first result
// rows.  *moved = false (and nothing changes) if the pool has no room for
// the plain form's region now.  The job's last batched launch has finished.
ea_status move_to_slabs(ea_server *s, ServerJob &j, int worker, bool *moved)
{
    *moved = false;
    const int L = j.h.job.L, n_tw = j.h.job.n_tw, n_meas = j.h.job.n_meas;
    const Layout lay = make_layout(L, n_tw, plain_rw(L));
    BatchJobHost nh = j.h;
    nh.RW = lay.RW;
    nh.W = lay.W;
    nh.POS = L * L * lay.RW;
    nh.bytes = align256(lay.total);
    size_t off = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->pool.alloc(nh.bytes, &off)) return EA_OK;
    }
    nh.base = s->pool_buf + off;
    auto give_back = [&](ea_sim *sim, ea_status st) {
        if (sim) ea_destroy(sim);
        std::lock_guard<std::mutex> lk(s->mu);
        s->pool.release(off, nh.bytes);
        return st;
    };
    const uint64_t t = j.h.t_host;
    std::vector<unsigned long long> results((size_t)n_meas * (size_t)j.h.obs_stride);
    if (!results.empty()) {
        const hipError_t e = hipMemcpy(results.data(), j.h.base + j.h.off_obs, 8 * results.size(),
                                       hipMemcpyDeviceToHost);
        if (e != hipSuccess) return give_back(nullptr, fail(EA_ERR_DEVICE, "hipMemcpy: %s", hipGetErrorString(e)));
    }
    ea_config c{};
    c.L = L;
    c.p = j.h.job.p;
    c.T = j.h.job.T;
    c.seed = j.h.job.seed;
    c.sample = j.h.job.sample;
    c.n_tw_slots = n_tw;
    c.stream = s->wstreams[(size_t)worker];
    c.dev_buf = nh.base;
    c.dev_buf_bytes = nh.bytes;
    c.words_per_row = nh.RW;
    ea_sim *sim = nullptr;
    ea_status st = ea_create_ex(&c, &sim);
    if (st != EA_OK) return give_back(nullptr, st);
    const size_t rep = 4 * 2 * (size_t)j.h.POS;  // bytes of one replica's two colour planes
    std::vector<int8_t> pm1((size_t)L * L * L);
    int next_tw = 0;
    while (next_tw < n_tw && j.h.tw[(size_t)next_tw] <= t) ++next_tw;
    for (int k = 0; k < next_tw && st == EA_OK; ++k) {
        for (int r = 0; r < 2 && st == EA_OK; ++r) {
            st = read_packed_pm1(j.h, j.h.base + j.h.off_snaps + ((size_t)k * 2 + (size_t)r) * rep, pm1.data(),
                                 s->stream);
            if (st == EA_OK) st = ea_set_spins(sim, r, pm1.data());
        }
        if (st == EA_OK) st = ea_set_time(sim, j.h.tw[(size_t)k]);
        if (st == EA_OK) st = ea_snapshot(sim, k);
    }
    for (int r = 0; r < 2 && st == EA_OK; ++r) {
        st = read_packed_pm1(j.h, j.h.base + j.h.off_spins + (size_t)r * rep, pm1.data(), s->stream);
        if (st == EA_OK) st = ea_set_spins(sim, r, pm1.data());
    }
    if (st == EA_OK) st = ea_set_time(sim, t);
    if (st == EA_OK) st = ea_sync(sim);
    if (st != EA_OK) return give_back(sim, st);
    int next_meas = 0;
    while (next_meas < n_meas && j.h.meas_t[(size_t)next_meas] <= t) ++next_meas;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->pool.release(j.pool_off, j.h.bytes);
    }
    j.pool_off = off;
    j.h = std::move(nh);
    j.sim = sim;
    j.streamed = true;
    j.worker = worker;
    j.results = std::move(results);
    j.next_meas = next_meas;
    j.next_tw = next_tw;
    j.sweep_s = 0.0;
    j.plan_K = 0;
    *moved = true;
    return EA_OK;
}

// One epoch: retire, admit, launch, wait.  Returns EA_OK with *progressed = 0
// when nothing was resident or admissible.
ea_status server_epoch(ea_server *s, int32_t *progressed)
{
    std::lock_guard<std::mutex> epoch_lock(s->epoch_mu);
    *progressed = 0;
    std::vector<ServerJob *> run;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        // admit in arrival order while memory and slots allow
        while (!s->pending.empty() && (int32_t)s->resident.size() < s->opts.max_resident) {
            ServerJob *j = s->pending.front().get();
            size_t off = 0;
            const BatchJobHost planned = j->h;
            bool restreamed = stream_small_job(s, *j);
            if (!s->pool.alloc(j->h.bytes, &off)) {
                if (!restreamed) break;
                j->h = planned;  // the batched form's region may still fit
                j->streamed = restreamed = false;
                if (!s->pool.alloc(j->h.bytes, &off)) break;
            }
            s->streamed_small += restreamed ? 1 : 0;
            j->pool_off = off;
            j->h.base = s->pool_buf + off;
            s->resident.push_back(std::move(s->pending.front()));
            s->pending.pop_front();
            s->state_of[j->id] = SJ_RUNNING;
            ++s->admitted;
            ea_status st;
            if (j->streamed) {
                ea_config c{};
                c.L = j->h.job.L;
                c.p = j->h.job.p;
                c.T = j->h.job.T;
                c.seed = j->h.job.seed;
                c.sample = j->h.job.sample;
                c.n_tw_slots = j->h.job.n_tw;
                // the worker with the least remaining work takes it, on its stream
                std::vector<double> load(s->wstreams.size(), 0.0);
                for (auto &r : s->resident)
                    if (r->streamed && r.get() != j)
                        load[(size_t)r->worker] += (double)r->h.job.L * r->h.job.L * r->h.job.L *
                                                   (double)(r->h.job.n_sweeps - r->h.t_host);
                j->worker = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                c.stream = s->wstreams[(size_t)j->worker];
                c.dev_buf = j->h.base;
                c.dev_buf_bytes = j->h.bytes;
                c.words_per_row = j->h.RW;  // the packing its footprint was planned with
                st = ea_create_ex(&c, &j->sim);
                if (st == EA_OK) server_slab_plan(*j, s->n_cu / (int)s->wstreams.size());
                j->results.assign((size_t)j->h.job.n_meas * (size_t)j->h.obs_stride, 0ull);
            } else {
                st = upload_schedule(j->h, s->stream);
                if (st == EA_OK) st = init_job_device(j->h, s->stream);
            }
            if (st != EA_OK) return st;
        }
        for (auto &p : s->resident) run.push_back(p.get());
    }
    if (run.empty()) return EA_OK;

    // a long batched job moves to the slab path when some worker has no job
    {
        std::vector<int> per_worker(s->wstreams.size(), 0);
        for (ServerJob *j : run)
            if (j->streamed) ++per_worker[(size_t)j->worker];
        const auto idle = std::find(per_worker.begin(), per_worker.end(), 0);
        ServerJob *best = nullptr;
        double best_rem = 0.0;
        for (ServerJob *j : run) {
            if (idle == per_worker.end() || j->streamed || !j->h.started || j->h.job.L < kLoneStreamL) continue;
            const double rem = (double)j->h.job.L * j->h.job.L * j->h.job.L * (double)(j->h.job.n_sweeps - j->h.t_host);
            if (rem >= kMoveMinSiteSweeps && rem > best_rem) {
                best = j;
                best_rem = rem;
            }
        }
        if (best) {
            bool moved = false;
            ea_status st = move_to_slabs(s, *best, (int)(idle - per_worker.begin()), &moved);
            if (st != EA_OK) return st;
            if (moved) {
                std::lock_guard<std::mutex> lk(s->mu);
                ++s->moved;
            }
        }
    }

    // spans: about opts.epoch_site_sweeps site-updates per replica, at least one sweep
    std::vector<BatchJobHost *> hs;
    std::vector<ServerJob *> batched, streamed;
    std::vector<uint64_t> span(run.size()), bspan;
    std::vector<ea::BatchJobDev> dj;
    for (size_t i = 0; i < run.size(); ++i) {
        ServerJob *j = run[i];
        if (j->streamed) {
            streamed.push_back(j);
            continue;
        }
        const uint64_t N = (uint64_t)j->h.job.L * j->h.job.L * j->h.job.L;
        const uint64_t want = std::max<uint64_t>(1, s->opts.epoch_site_sweeps / N);
        span[i] = std::min<uint64_t>(want, j->h.job.n_sweeps - j->h.t_host);
        batched.push_back(j);
        bspan.push_back(span[i]);
        hs.push_back(&j->h);
        dj.push_back(make_job_dev(j->h));
    }
    const auto t0 = steady::now();
    if (!batched.empty()) {
        size_t lds = 0;
        for (BatchJobHost *h : hs) lds = std::max(lds, (size_t)batch_lds_words(h->job.L, h->RW) * 4);
        std::vector<ea::BatchUnit> units;
        order_units(hs, bspan, units);
        debug_order_units(hs.data(), units);
        for (auto &u : units) {
            const BatchJobHost &h = *hs[(size_t)u.job];
            u.t_stop = (uint32_t)(h.t_host + bspan[(size_t)u.job]);
            u.first = h.started ? 0 : 1;
        }
        EA_HIP(hipMemcpyAsync(s->d_jobs, dj.data(), sizeof(ea::BatchJobDev) * dj.size(), hipMemcpyHostToDevice,
                              s->stream));
        EA_HIP(hipMemcpyAsync(s->d_units, units.data(), sizeof(ea::BatchUnit) * units.size(),
                              hipMemcpyHostToDevice, s->stream));
        EA_HIP(hipEventRecord(s->ev_batch[0], s->stream));
        hipLaunchKernelGGL(ea::batch_kernel, dim3((unsigned)units.size()), dim3(ea::kBatchThreads), lds, s->stream,
                           s->d_jobs, s->d_units, debug_poison_word(), (int)(lds / 4));
        EA_HIP(hipGetLastError());
        EA_HIP(hipEventRecord(s->ev_batch[1], s->stream));
    }
    // streamed jobs, on their workers' streams: one host thread per worker
    // with jobs, each thread's jobs splitting the expected epoch time
    if (!streamed.empty()) {
        // The streamed phase gets the batched launch's time scaled by the
        // ratio of the streamed jobs' remaining site-updates to the batched
        // jobs', between 1x and 16x (and at least 2 ms): both forms then
        // progress in proportion to their work.
        double rem_streamed = 0.0, rem_batched = 0.0;
        for (ServerJob *j : run) {
            const double N = (double)j->h.job.L * j->h.job.L * j->h.job.L;
            const double rem = N * (double)(j->h.job.n_sweeps - j->h.t_host);
            (j->streamed ? rem_streamed : rem_batched) += rem;
        }
        const double ratio = rem_batched > 0.0 ? std::min(16.0, std::max(1.0, rem_streamed / rem_batched)) : 16.0;
        const double target = std::max(s->last_batch_s * ratio, 2e-3);
        // each worker's jobs, in admission order, on its stream
        std::vector<std::vector<size_t>> lists;
        {
            std::vector<std::vector<size_t>> by_worker(s->wstreams.size());
            for (size_t i = 0; i < run.size(); ++i)
                if (run[i]->streamed) by_worker[(size_t)run[i]->worker].push_back(i);
            for (auto &l : by_worker)
                if (!l.empty()) lists.push_back(std::move(l));
        }
        const int n_workers = (int)lists.size();
        // Plans of this epoch: the workers with jobs share the compute units
        // that the batched launch leaves free, so that they can start beside
        // it; where it leaves fewer than a quarter, they wait for it and
        // share all of them.  (Plans never change results.)
        const int busy = batched.empty() ? 0 : (int)(2 * batched.size());
        const bool overlap = busy > 0 && 4 * (s->n_cu - busy) >= s->n_cu;
        const int share = (overlap ? s->n_cu - busy : s->n_cu) / n_workers;
        for (auto &l : lists)
            for (size_t i : l) server_slab_plan(*run[i], share);
        std::vector<std::string> errs((size_t)n_workers);
        auto advance = [&](int k) {
            (void)hipSetDevice(s->device);
            // unless the plans leave the batched launch its compute units,
            // after it: slab workgroups that became resident beside it would
            // wait for its CUs (and the per-sweep timing below would include
            // that wait)
            if (!batched.empty() && !overlap && hipEventSynchronize(s->ev_batch[1]) != hipSuccess) {
                errs[(size_t)k] = "hipEventSynchronize failed";
                return;
            }
            const double budget = target / (double)lists[(size_t)k].size();
            for (size_t i : lists[(size_t)k]) {
                ServerJob *j = run[i];
                const double per_sweep = j->sweep_s > 0.0 ? j->sweep_s : 2e-5;
                const uint64_t want = (uint64_t)std::max(1.0, std::floor(budget / per_sweep));
                span[i] = std::min<uint64_t>(want, j->h.job.n_sweeps - j->h.t_host);
                const auto a = steady::now();
                ea_status st = server_advance_streamed(*j, j->h.t_host + span[i]);
                if (st == EA_OK) st = ea_sync(j->sim);
                if (st != EA_OK) {
                    errs[(size_t)k] = ea_last_error();
                    return;
                }
                if (span[i] > 0) {
                    const double per = std::chrono::duration<double>(steady::now() - a).count() / (double)span[i];
                    j->sweep_s = j->sweep_s > 0.0 ? 0.5 * (j->sweep_s + per) : per;
                }
            }
        };
        std::vector<std::thread> helpers;
        std::vector<int> here = {0};  // lists this thread advances itself
        for (int k = 1; k < n_workers; ++k) {
            try {
                helpers.emplace_back(advance, k);
            } catch (const std::exception &) {
                here.push_back(k);  // no thread to spare: run the list here
            }
        }
        for (int k : here) advance(k);
        for (auto &h : helpers) h.join();
        for (const std::string &e : errs)
            if (!e.empty()) return fail(EA_ERR_DEVICE, "streamed job: %s", e.c_str());
    }
    EA_HIP(hipStreamSynchronize(s->stream));
    if (!batched.empty()) {
        float ms = 0.0f;
        EA_HIP(hipEventElapsedTime(&ms, s->ev_batch[0], s->ev_batch[1]));
        s->last_batch_s = 1e-3 * (double)ms;
    }
    const auto t1 = steady::now();

    // bookkeeping; finished jobs hand their results over and free their memory
    double epoch_flips = 0.0;
    std::vector<ServerJob *> finished;
    for (size_t i = 0; i < run.size(); ++i) {
        BatchJobHost &h = run[i]->h;
        h.t_host += span[i];
        h.started = true;
        epoch_flips += 2.0 * h.job.L * h.job.L * h.job.L * (double)span[i];
        if (h.t_host >= h.job.n_sweeps) finished.push_back(run[i]);
    }
    for (ServerJob *j : finished) {
        if (j->streamed) {  // results were taken at each measurement
            ea_destroy(j->sim);
            j->sim = nullptr;
            continue;
        }
        j->results.resize((size_t)j->h.job.n_meas * (size_t)j->h.obs_stride);
        if (!j->results.empty())
            EA_HIP(hipMemcpy(j->results.data(), j->h.base + j->h.off_obs, 8 * j->results.size(),
                             hipMemcpyDeviceToHost));
    }
    const auto t2 = steady::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->epochs;
        s->flips += epoch_flips;
        s->busy_s += std::chrono::duration<double>(t1 - t0).count();
        for (ServerJob *j : finished) {
            j->t_done = t2;
            s->latencies.push_back(std::chrono::duration<double>(j->t_done - j->t_submit).count());
            s->pool.release(j->pool_off, j->h.bytes);
            j->h.base = nullptr;
            auto it = std::find_if(s->resident.begin(), s->resident.end(),
                                   [&](const std::unique_ptr<ServerJob> &p) { return p.get() == j; });
            s->state_of[j->id] = SJ_DONE;
            ++s->completed;
            s->done[j->id] = std::move(*it);
            s->resident.erase(it);
        }
    }
    s->cv.notify_all();
    *progressed = 1;
    return EA_OK;
}

void server_worker(ea_server *s)
{
    (void)hipSetDevice(s->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stop || !s->pending.empty() || !s->resident.empty(); });
            if (s->stop) return;
        }
        int32_t progressed = 0;
        ea_status st = server_epoch(s, &progressed);
        if (st != EA_OK) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->worker_error = ea_last_error();
            s->stop = true;
            s->cv.notify_all();
            return;
        }
        if (!progressed) {
            // nothing admissible right now (memory full with nothing resident cannot happen)
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
}

double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

}  // namespace

extern "C" {

ea_status ea_server_create(const ea_server_opts *opts, ea_server **out)
{
    if (!opts || !out) return fail(EA_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (opts->hbm_budget < 4096) return fail(EA_ERR_ARG, "hbm_budget %zu is too small", opts->hbm_budget);
    if (opts->max_resident < 1 || opts->max_resident > 4096)
        return fail(EA_ERR_ARG, "max_resident %d outside [1, 4096]", opts->max_resident);
    if (opts->max_pending < 1) return fail(EA_ERR_ARG, "max_pending must be positive");
    ea_server *s = new (std::nothrow) ea_server();
    if (!s) return fail(EA_ERR_NOMEM, "host allocation failed");
    s->opts = *opts;
    if (!s->opts.epoch_site_sweeps) s->opts.epoch_site_sweeps = 64ull * 64 * 64 * 64;
    s->lds_bytes = (size_t)batch_lds_words(ea::kBatchMaxL, ea::words_per_row_c(ea::kBatchMaxL / 2)) * 4;
    ea_status st = prepare_batch_lds(s->lds_bytes);
    hipError_t e = hipGetDevice(&s->device);
    if (st == EA_OK && e != hipSuccess) st = fail(EA_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (st != EA_OK) {
        delete s;
        return st;
    }
    if (opts->stream) {
        s->stream = (hipStream_t)opts->stream;
    } else {
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete s;
            return fail(EA_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        s->own_stream = true;
    }
    e = hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, s->device);
    if (e != hipSuccess) {
        ea_server_destroy(s);
        return fail(EA_ERR_DEVICE, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
    }
    s->wstreams.assign((size_t)server_stream_workers(), nullptr);
    for (hipStream_t &ws : s->wstreams) {
        e = hipStreamCreateWithFlags(&ws, hipStreamNonBlocking);
        if (e != hipSuccess) {
            ws = nullptr;
            ea_server_destroy(s);
            return fail(EA_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
    }
    for (int k = 0; k < 2; ++k) {
        e = hipEventCreate(&s->ev_batch[k]);
        if (e != hipSuccess) {
            ea_server_destroy(s);
            return fail(EA_ERR_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    const size_t table_bytes = align256(sizeof(ea::BatchJobDev) * (size_t)opts->max_resident) +
                               align256(sizeof(ea::BatchUnit) * 2 * (size_t)opts->max_resident);
    e = hipMalloc((void **)&s->pool_buf, align256(opts->hbm_budget) + table_bytes);
    if (e != hipSuccess) {
        ea_server_destroy(s);
        return fail(EA_ERR_NOMEM, "hipMalloc(%zu): %s", opts->hbm_budget, hipGetErrorString(e));
    }
    s->pool.reset(align256(opts->hbm_budget));
    s->d_jobs = (ea::BatchJobDev *)(s->pool_buf + align256(opts->hbm_budget));
    s->d_units = (ea::BatchUnit *)((char *)s->d_jobs +
                                   align256(sizeof(ea::BatchJobDev) * (size_t)opts->max_resident));
    *out = s;
    return EA_OK;
}

void ea_server_destroy(ea_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto &j : s->resident)
        if (j->sim) ea_destroy(j->sim);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->pool_buf) (void)hipFree(s->pool_buf);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    for (hipStream_t ws : s->wstreams)
        if (ws) (void)hipStreamDestroy(ws);
    for (hipEvent_t ev : s->ev_batch)
        if (ev) (void)hipEventDestroy(ev);
    delete s;
}

ea_status ea_server_footprint(const ea_job *job, size_t *bytes)
{
    if (!job || !bytes) return fail(EA_ERR_ARG, "NULL argument");
    ServerJob j;
    ea_status st = plan_server_job(*job, j);
    if (st != EA_OK) return st;
    *bytes = j.h.bytes;
    return EA_OK;
}

ea_status ea_server_submit(ea_server *s, const ea_job *job, uint64_t *id)
{
    if (!s || !job || !id) return fail(EA_ERR_ARG, "NULL argument");
    auto j = std::make_unique<ServerJob>();
    ea_status st = plan_server_job(*job, *j);
    if (st != EA_OK) return st;
    if (align256(j->h.bytes) > s->pool.size)
        return fail(EA_ERR_ARG, "job needs %zu bytes, more than the whole budget %zu", j->h.bytes, s->pool.size);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->worker_error.empty()) return fail(EA_ERR_STATE, "worker stopped: %s", s->worker_error.c_str());
        if ((int32_t)s->pending.size() >= s->opts.max_pending)
            return fail(EA_ERR_BUSY, "%zu jobs already wait", s->pending.size());
        j->id = s->next_id++;
        j->t_submit = steady::now();
        if (!s->have_first) {
            s->have_first = true;
            s->first_submit = j->t_submit;
        }
        *id = j->id;
        s->state_of[j->id] = SJ_PENDING;
        ++s->submitted;
        s->pending.push_back(std::move(j));
    }
    s->cv.notify_all();
    return EA_OK;
}

ea_status ea_server_step(ea_server *s, int32_t *progressed)
{
    if (!s || !progressed) return fail(EA_ERR_ARG, "NULL argument");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->worker_on) return fail(EA_ERR_STATE, "a worker thread runs the epochs");
    }
    return server_epoch(s, progressed);
}

ea_status ea_server_start(ea_server *s)
{
    if (!s) return fail(EA_ERR_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->worker_on) return EA_OK;
    s->stop = false;
    s->worker_on = true;
    s->worker = std::thread(server_worker, s);
    return EA_OK;
}

ea_status ea_server_stop(ea_server *s)
{
    if (!s) return fail(EA_ERR_ARG, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->worker_on) return EA_OK;
        s->stop = true;
    }
    s->cv.notify_all();
    s->worker.join();
    std::lock_guard<std::mutex> lk(s->mu);
    s->worker_on = false;
    s->stop = false;
    if (!s->worker_error.empty()) return fail(EA_ERR_DEVICE, "worker failed: %s", s->worker_error.c_str());
    return EA_OK;
}

ea_status ea_server_drain(ea_server *s, double timeout_s)
{
    if (!s) return fail(EA_ERR_ARG, "server is NULL");
    bool threaded;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        threaded = s->worker_on;
    }
    const auto deadline = steady::now() + std::chrono::duration_cast<steady::duration>(
                                              std::chrono::duration<double>(timeout_s));
    if (!threaded) {
        for (;;) {
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (s->pending.empty() && s->resident.empty()) return EA_OK;
            }
            if (steady::now() > deadline) return fail(EA_ERR_BUSY, "drain timed out");
            int32_t progressed = 0;
            ea_status st = server_epoch(s, &progressed);
            if (st != EA_OK) return st;
        }
    }
    std::unique_lock<std::mutex> lk(s->mu);
    const bool ok = s->cv.wait_until(lk, deadline, [&] {
        return (s->pending.empty() && s->resident.empty()) || !s->worker_error.empty();
    });
    if (!s->worker_error.empty()) return fail(EA_ERR_DEVICE, "worker failed: %s", s->worker_error.c_str());
    return ok ? EA_OK : fail(EA_ERR_BUSY, "drain timed out");
}

ea_status ea_server_poll(ea_server *s, uint64_t id, int32_t *state)
{
    if (!s || !state) return fail(EA_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->state_of.find(id);
    if (it == s->state_of.end()) return fail(EA_ERR_ARG, "unknown job id %llu", (unsigned long long)id);
    *state = it->second;
    return EA_OK;
}

ea_status ea_server_result(ea_server *s, uint64_t id, int32_t k, ea_obs *out)
{
    if (!s || !out) return fail(EA_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->done.find(id);
    if (it == s->done.end()) {
        if (s->state_of.count(id)) return fail(EA_ERR_STATE, "job %llu has not finished", (unsigned long long)id);
        return fail(EA_ERR_ARG, "unknown job id %llu", (unsigned long long)id);
    }
    const ServerJob &j = *it->second;
    if (k < 0 || k >= j.h.job.n_meas) return fail(EA_ERR_ARG, "measurement %d out of range", k);
    return fill_obs(j.h, j.results.data() + (size_t)k * (size_t)j.h.obs_stride, k, out);
}

ea_status ea_server_latency(ea_server *s, uint64_t id, double *seconds)
{
    if (!s || !seconds) return fail(EA_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->done.find(id);
    if (it == s->done.end()) return fail(EA_ERR_STATE, "job %llu has not finished", (unsigned long long)id);
    *seconds = std::chrono::duration<double>(it->second->t_done - it->second->t_submit).count();
    return EA_OK;
}

ea_status ea_server_release(ea_server *s, uint64_t id)
{
    if (!s) return fail(EA_ERR_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->done.find(id);
    if (it == s->done.end()) return fail(EA_ERR_STATE, "job %llu has not finished", (unsigned long long)id);
    s->done.erase(it);
    s->state_of.erase(id);
    return EA_OK;
}

ea_status ea_server_stats(ea_server *s, ea_server_report *out)
{
    if (!s || !out) return fail(EA_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    ea_server_report r{};
    r.submitted = s->submitted;
    r.admitted = s->admitted;
    r.completed = s->completed;
    r.resident = (int32_t)s->resident.size();
    r.pending = (int32_t)s->pending.size();
    r.epochs = s->epochs;
    r.p50_latency_s = percentile(s->latencies, 0.50);
    r.p99_latency_s = percentile(s->latencies, 0.99);
    r.max_latency_s = s->latencies.empty() ? 0.0 : *std::max_element(s->latencies.begin(), s->latencies.end());
    double sum = 0.0;
    for (double v : s->latencies) sum += v;
    r.mean_latency_s = s->latencies.empty() ? 0.0 : sum / (double)s->latencies.size();
    r.flips = s->flips;
    r.busy_s = s->busy_s;
    r.wall_s = s->have_first ? std::chrono::duration<double>(steady::now() - s->first_submit).count() : 0.0;
    r.ps_per_flip = s->flips > 0 ? s->busy_s / s->flips * 1e12 : 0.0;
    r.hbm_in_use = s->pool.in_use;
    r.hbm_peak = s->pool.peak;
    r.streamed_small = s->streamed_small;
    r.moved = s->moved;
    *out = r;
    return EA_OK;
}

}  // extern "C"
