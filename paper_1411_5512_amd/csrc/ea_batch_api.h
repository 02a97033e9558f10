// ea_batch_api.h -- host side of the batched form (ea_batch_* in ea.h) and
// the per-job helpers the serving loop shares with it.  Included once, at the
// end of ea_api.hip, so that the whole library is one translation unit.
#pragma once

#include <cstdlib>
#include <map>
#include <mutex>
#include <numeric>
#include <queue>
#include <type_traits>

namespace {

// Host record of one job of the batched kernel: parameters, schedule,
// geometry and the layout of its device region (offsets from `base`).
// Launch configuration of one lattice size: row packing, working threads
// per workgroup and threshold-select variant (chosen by the autotuner).
struct TuneCfg {
    int rw = 0, nt = 0, sel = 0;
};

int round_up64(int v) { return (v + 63) / 64 * 64; }

TuneCfg default_cfg(int L)
{
    TuneCfg c;
    c.rw = ea::words_per_row_c(L / 2);
    c.nt = std::min(ea::kBatchThreads, round_up64(L * L * c.rw));
    c.sel = ea::SEL_LDS;
    return c;
}

bool cfg_valid(int L, const TuneCfg &c)
{
    const int R = L / 2, rw0 = ea::words_per_row_c(R), rw1 = ea::finer_words_per_row_c(R, rw0);
    if (c.rw != rw0 && (rw1 == 0 || c.rw != rw1)) return false;
    if (c.nt < 64 || c.nt > ea::kBatchThreads || c.nt % 64) return false;
    if (c.nt < L * c.rw) return false;  // every thread owns at least one column of a z-plane
    return c.sel == ea::SEL_LDS || c.sel == ea::SEL_REG;
}

struct BatchJobHost {
    ea_job job{};             // parameters (schedule pointers not kept)
    TuneCfg cfg;
    std::vector<uint32_t> meas_t, tw;
    int R = 0, RW = 0, W = 0, POS = 0, obs_stride = 0;
    uint32_t thr[3] = {0, 0, 0};
    uint64_t pcut = 0;
    size_t off_spins = 0, off_bonds = 0, off_snaps = 0, off_mspins = 0, off_obs = 0, off_arrive = 0,
           off_tnow = 0, off_pub = 0, off_xbuf = 0, off_meas_t = 0, off_tw = 0, bytes = 0;
    int parts = 1;            // workgroups per replica (2: split into z-slabs)
    uint32_t *err = nullptr;  // device word a split pair sets when it gives up waiting
    char *base = nullptr;     // device region of this job
    uint64_t t_host = 0;      // sweeps done (host mirror)
    bool started = false;     // a span has run (events at t = 0 are taken)
};

bool batch_L_ok(int L) { return L >= 8 && L <= ea::kBatchMaxL && L % 8 == 0; }

int batch_lds_words(int L, int rw) { return 8 * L * L * rw + 16; }

// LDS of one slab of a split replica: its half of the lattice, the z
// couplings of the plane below it and the broadcast words.
int slab_lds_words(int L, int rw) { return 8 * (L / 2) * L * rw + 2 * L * rw + 16; }

int job_lds_words(const BatchJobHost &h)
{
    return h.parts == 2 ? slab_lds_words(h.job.L, h.RW) : batch_lds_words(h.job.L, h.RW);
}

ea_status copy_schedule(const uint64_t *src, int32_t n, uint64_t n_sweeps, const char *what,
                        std::vector<uint32_t> &dst)
{
    dst.clear();
    if (n < 0) return fail(EA_ERR_ARG, "%s count %d is negative", what, n);
    if (n > 0 && !src) return fail(EA_ERR_ARG, "%s is NULL", what);
    for (int32_t i = 0; i < n; ++i) {
        if (src[i] > n_sweeps) return fail(EA_ERR_ARG, "%s[%d]=%llu beyond %llu sweeps", what, i,
                                            (unsigned long long)src[i], (unsigned long long)n_sweeps);
        if (i > 0 && src[i] <= src[i - 1]) return fail(EA_ERR_ARG, "%s is not strictly increasing", what);
        dst.push_back((uint32_t)src[i]);
    }
    return EA_OK;
}

// Checks and host data shared by both kinds of job: parameters, schedules,
// thresholds, coupling cut and the size of one measurement's counters.
ea_status plan_common(const ea_job &in, int index, BatchJobHost &h)
{
    if (!(in.p >= 0.0 && in.p <= 1.0)) return fail(EA_ERR_ARG, "job %d: p=%g outside [0, 1]", index, in.p);
    if (!(in.T >= 0.0) || !std::isfinite(in.T))
        return fail(EA_ERR_ARG, "job %d: T=%g must be finite and >= 0", index, in.T);
    if (in.n_sweeps >= (1ull << 32)) return fail(EA_ERR_ARG, "job %d: n_sweeps must be below 2^32", index);
    if (in.n_tw > kMaxSlots) return fail(EA_ERR_ARG, "job %d: n_tw=%d above %d", index, in.n_tw, kMaxSlots);
    ea_status st = copy_schedule(in.meas_t, in.n_meas, in.n_sweeps, "meas_t", h.meas_t);
    if (st == EA_OK) st = copy_schedule(in.tw, in.n_tw, in.n_sweeps, "tw", h.tw);
    if (st != EA_OK) return st;
    h.job = in;
    h.job.meas_t = nullptr;
    h.job.tw = nullptr;
    h.R = in.L / 2;
    h.obs_stride = ea::M_AUTO + 2 * in.n_tw + 3 * (h.R + 1);
    host_thresholds(in.T, h.thr);
    h.pcut = (uint64_t)std::floor(std::ldexp(in.p, 32));
    return EA_OK;
}

// Validate a job of the batched kernel and lay out its device region
// (offsets from 0).
ea_status plan_job(const ea_job &in, int index, BatchJobHost &h, const TuneCfg *cfg = nullptr)
{
    if (!batch_L_ok(in.L))
        return fail(EA_ERR_ARG, "job %d: L=%d must be a multiple of 8 in [8, %d] for the batched form", index,
                    in.L, ea::kBatchMaxL);
    ea_status st = plan_common(in, index, h);
    if (st != EA_OK) return st;
    h.cfg = cfg ? *cfg : default_cfg(in.L);
    if (!cfg_valid(in.L, h.cfg))
        return fail(EA_ERR_ARG, "job %d: invalid launch configuration rw=%d nt=%d sel=%d", index, h.cfg.rw,
                    h.cfg.nt, h.cfg.sel);
    h.RW = h.cfg.rw;
    h.W = h.R / h.RW;
    h.POS = in.L * in.L * h.RW;
    const size_t spin4 = 4 * (size_t)h.POS;  // words of [replica][colour]
    size_t off = 0;
    h.off_spins = off;
    off += 4 * spin4;
    h.off_bonds = off = align256(off);
    off += 4 * 6 * (size_t)h.POS;
    h.off_snaps = off = align256(off);
    off += 4 * spin4 * (size_t)in.n_tw;
    h.off_mspins = off = align256(off);
    off += 4 * spin4 * (size_t)in.n_meas;
    h.off_obs = off = align256(off);
    off += 8 * (size_t)in.n_meas * (size_t)h.obs_stride;
    h.off_arrive = off = align256(off);
    off += 4 * (size_t)in.n_meas;
    h.off_tnow = off;
    off += 8;
    h.off_pub = off = align256(off);
    off += 8 * 4;
    h.off_xbuf = off = align256(off);
    off += 4 * 32 * (size_t)in.L * (size_t)h.RW;
    h.off_meas_t = off = align256(off);
    off += 4 * (size_t)in.n_meas;
    h.off_tw = off = align256(off);
    off += 4 * (size_t)in.n_tw;
    h.bytes = align256(off);
    return EA_OK;
}

// A job whose lattice does not fit one workgroup's LDS: it runs through the
// plain form's HBM-streaming kernels in the plain form's device layout, so
// its region is what ea_footprint gives.
ea_status plan_streamed_job(const ea_job &in, int index, BatchJobHost &h)
{
    if (!valid_L(in.L) || batch_L_ok(in.L))
        return fail(EA_ERR_ARG, "job %d: L=%d is not a streamed size (multiple of 8 in (%d, %d])", index, in.L,
                    ea::kBatchMaxL, kMaxL);
    ea_status st = plan_common(in, index, h);
    if (st != EA_OK) return st;
    const Layout lay = make_layout(in.L, in.n_tw, plain_rw(in.L));
    h.RW = lay.RW;
    h.W = lay.W;
    h.POS = in.L * in.L * h.RW;
    h.bytes = align256(lay.total);
    return EA_OK;
}

ea::BatchJobDev make_job_dev(const BatchJobHost &h)
{
    ea::BatchJobDev d{};
    d.L = h.job.L;
    d.rw = h.cfg.rw;
    d.nt = h.cfg.nt;
    d.sel = h.cfg.sel;
    d.k0 = (uint32_t)(h.job.seed & 0xffffffffu);
    d.k1 = (uint32_t)(h.job.seed >> 32);
    d.sample = h.job.sample;
    d.thr1 = h.thr[0];
    d.thr2 = h.thr[1];
    d.thr3 = h.thr[2];
    d.n_meas = h.job.n_meas;
    d.n_tw = h.job.n_tw;
    d.obs_stride = h.obs_stride;
    d.spins = (uint32_t *)(h.base + h.off_spins);
    d.bonds = (const uint32_t *)(h.base + h.off_bonds);
    d.snaps = (uint32_t *)(h.base + h.off_snaps);
    d.mspins = (uint32_t *)(h.base + h.off_mspins);
    d.meas_t = (const uint32_t *)(h.base + h.off_meas_t);
    d.tw_t = (const uint32_t *)(h.base + h.off_tw);
    d.obs = (unsigned long long *)(h.base + h.off_obs);
    d.arrive = (uint32_t *)(h.base + h.off_arrive);
    d.t_now = (uint32_t *)(h.base + h.off_tnow);
    d.parts = h.parts;
    d.pub = (unsigned long long *)(h.base + h.off_pub);
    d.xbuf = (uint32_t *)(h.base + h.off_xbuf);
    d.err = h.err;
    return d;
}

// Copy the schedule to the job's region (the host vectors stay alive with h).
ea_status upload_schedule(const BatchJobHost &h, hipStream_t stream)
{
    if (!h.meas_t.empty())
        EA_HIP(hipMemcpyAsync(h.base + h.off_meas_t, h.meas_t.data(), 4 * h.meas_t.size(), hipMemcpyHostToDevice,
                              stream));
    if (!h.tw.empty())
        EA_HIP(hipMemcpyAsync(h.base + h.off_tw, h.tw.data(), 4 * h.tw.size(), hipMemcpyHostToDevice, stream));
    return EA_OK;
}

// Generate the job's couplings and initial spins and clear its counters.
ea_status init_job_device(BatchJobHost &h, hipStream_t stream)
{
    ea::Lattice lat;
    lat.spins = (uint32_t *)(h.base + h.off_spins);
    lat.bonds = (uint32_t *)(h.base + h.off_bonds);
    ea::Geom g;
    g.L = h.job.L;
    g.R = h.R;
    g.RW = h.RW;
    g.rows = h.job.L * h.job.L;
    g.plane = h.POS;
    ea_status st = launch_init_lattice(lat, g, h.W, h.job.seed, h.job.sample, h.pcut, stream);
    if (st != EA_OK) return st;
    const size_t n_obs = (size_t)h.job.n_meas * (size_t)h.obs_stride;
    if (n_obs)
        hipLaunchKernelGGL(ea::zero_u64_kernel, dim3(blocks_for(n_obs)), dim3(256), 0, stream,
                           (unsigned long long *)(h.base + h.off_obs), n_obs);
    // arrive[n_meas] and t_now[2] are contiguous 32-bit words
    const size_t n_ctl32 = (size_t)h.job.n_meas + 2;
    hipLaunchKernelGGL(ea::zero_u32_kernel, dim3(blocks_for(n_ctl32)), dim3(256), 0, stream,
                       (uint32_t *)(h.base + h.off_arrive), n_ctl32);
    hipLaunchKernelGGL(ea::zero_u64_kernel, dim3(1), dim3(256), 0, stream,
                       (unsigned long long *)(h.base + h.off_pub), (size_t)4);
    EA_HIP(hipGetLastError());
    h.t_host = 0;
    h.started = false;
    return EA_OK;
}

// Turn measurement k's popcount counters m[obs_stride] into an ea_obs.
ea_status fill_obs(const BatchJobHost &h, const unsigned long long *m, int32_t k, ea_obs *out)
{
    if (out->autocorr && out->n_tw != h.job.n_tw)
        return fail(EA_ERR_ARG, "n_tw=%d but the job has %d snapshot times", out->n_tw, h.job.n_tw);
    if (out->c4 && out->rmax != h.R) return fail(EA_ERR_ARG, "rmax=%d but L/2=%d", out->rmax, h.R);
    const int64_t N = (int64_t)h.job.L * h.job.L * h.job.L;
    const uint32_t t = h.meas_t[(size_t)k];
    out->t = t;
    for (int r = 0; r < 2; ++r) {
        out->unsat[r] = (int64_t)m[ea::M_UNSAT + r];
        out->mag[r] = N - 2 * (int64_t)m[ea::M_DOWN + r];
    }
    out->overlap = N - 2 * (int64_t)m[ea::M_QDIFF];
    if (out->autocorr) {
        for (int r = 0; r < 2; ++r)
            for (int s = 0; s < h.job.n_tw; ++s)
                out->autocorr[r * h.job.n_tw + s] =
                    h.tw[(size_t)s] <= t ? N - 2 * (int64_t)m[ea::M_AUTO + 2 * s + r] : 0;
        if (out->tw)
            for (int s = 0; s < h.job.n_tw; ++s) out->tw[s] = h.tw[(size_t)s] <= t ? h.tw[(size_t)s] : 0;
    }
    if (out->c4) {
        const int base = ea::M_AUTO + 2 * h.job.n_tw;
        for (int i = 0; i < 3 * (h.R + 1); ++i) out->c4[i] = N - 2 * (int64_t)m[base + i];
    }
    return EA_OK;
}

// Canonical +-1 spins of one configuration in the job's packed layout
// ([colour][POS] words at dev).
ea_status read_packed_pm1(const BatchJobHost &h, const char *dev, int8_t *pm1, hipStream_t stream)
{
    std::vector<uint32_t> words(2 * (size_t)h.POS);
    EA_HIP(hipMemcpyAsync(words.data(), dev, 4 * words.size(), hipMemcpyDeviceToHost, stream));
    EA_HIP(hipStreamSynchronize(stream));
    Layout y = make_layout(h.job.L, 0, h.RW);
    const int64_t N = (int64_t)h.job.L * h.job.L * h.job.L;
    for (int64_t i = 0; i < N; ++i) {
        SiteAddr a = address_of(y, i);
        const uint32_t bit = (words[(size_t)a.c * h.POS + a.word] >> a.bit) & 1u;
        pm1[i] = bit ? (int8_t)-1 : (int8_t)1;
    }
    return EA_OK;
}

// Replica r's current spins as int8 +-1.
ea_status read_job_spins(const BatchJobHost &h, int32_t r, int8_t *pm1, hipStream_t stream)
{
    return read_packed_pm1(h, h.base + h.off_spins + 4 * (size_t)r * 2 * h.POS, pm1, stream);
}

// Check that a launch with this much dynamic LDS fits one workgroup, and
// allow it (the kernel's default cap is lower).
// The kernel's dynamic-LDS limit only ever grows, so that a batch created
// later with smaller jobs does not lower it under one that still runs.
std::mutex g_lds_mu;
size_t g_lds_attr = 0;

ea_status prepare_batch_lds(size_t dyn_bytes)
{
    int dev = 0, lds_limit = 0;
    EA_HIP(hipGetDevice(&dev));
    EA_HIP(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (dyn_bytes + 4 * (size_t)ea::kSelectTableWords > (size_t)lds_limit)
        return fail(EA_ERR_ARG, "the largest job needs %zu bytes of LDS, the device offers %d", dyn_bytes,
                    lds_limit);
    std::lock_guard<std::mutex> lk(g_lds_mu);
    if (dyn_bytes > g_lds_attr) {
        EA_HIP(hipFuncSetAttribute((const void *)ea::batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)dyn_bytes));
        g_lds_attr = dyn_bytes;
    }
    return EA_OK;
}

// Units of a set of jobs.  Split replicas come first, largest first, as
// (slab 0, slab 1) pairs at even positions, so that the two workgroups of a
// pair sit at the same position of the in-order dispatch on their XCDs and
// are resident together; then the other units, largest remaining work first
// (the longest units start first), the two replicas of a job adjacent so that
// they reach each measurement at about the same time.
void order_units(const std::vector<BatchJobHost *> &jobs, const std::vector<uint64_t> &span,
                 std::vector<ea::BatchUnit> &units)
{
    std::vector<int32_t> order(jobs.size());
    std::iota(order.begin(), order.end(), 0);
    auto work = [&](int32_t a) {
        const double L = (double)jobs[(size_t)a]->job.L;
        return L * L * L * (double)span[(size_t)a];
    };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
        const int pa = jobs[(size_t)a]->parts, pc = jobs[(size_t)c]->parts;
        if (pa != pc) return pa > pc;
        return work(a) > work(c);
    });
    units.clear();
    for (int32_t j : order)
        for (int32_t r = 0; r < 2; ++r)
            for (int32_t k = 0; k < jobs[(size_t)j]->parts; ++k) units.push_back(ea::BatchUnit{j, r, 0u, 1, k});
}

// The debug order (ea_set_debug) of a unit list made by order_units: the
// split pairs among themselves (each pair kept together, so that all of them
// are still dispatched, and resident, first) and the whole replicas among
// themselves.  jobs: indexed by BatchUnit::job.
template <class JobRef>
void debug_order_units(const JobRef *jobs, std::vector<ea::BatchUnit> &units)
{
    if (debug_grid_order() == 0) return;
    auto parts = [&](const ea::BatchUnit &u) {
        if constexpr (std::is_pointer<JobRef>::value) return jobs[u.job]->parts;
        else return jobs[u.job].parts;
    };
    size_t n_split = 0;
    while (n_split < units.size() && parts(units[n_split]) > 1) ++n_split;
    std::vector<std::pair<ea::BatchUnit, ea::BatchUnit>> pairs;
    for (size_t i = 0; i + 1 < n_split; i += 2) pairs.push_back({units[i], units[i + 1]});
    debug_permute(pairs.data(), pairs.size());
    for (size_t i = 0; i < pairs.size(); ++i) {
        units[2 * i] = pairs[i].first;
        units[2 * i + 1] = pairs[i].second;
    }
    debug_permute(units.data() + n_split, units.size() - n_split);
}

// Which jobs to split.  For each size threshold (none, 64, 56, 48) whose
// slabs all fit the device at once (one per CU, so that both workgroups of
// every pair are dispatched at the start), the in-order dispatch of the
// resulting unit list onto n_cu one-unit CUs is simulated and the threshold
// with the shortest estimated makespan is kept.  Time model per half-step
// (measured on MI355X): a whole replica takes kHalfStepL64 (L/64)^kSizeExp
// (smaller lattices use a CU less fully than the site count alone says); a
// slab takes half of that plus kSlabExchange, but at least kSlabFloor, the
// latency of the boundary exchange (wait, remote reads, publication).  Only
// jobs in their default launch configuration (the slab kernel exists for
// that one) split.
constexpr double kHalfStepL64 = 12.6e-6;
constexpr double kSizeExp = 2.57;  // L = 48 measured at 0.478 of L = 64
constexpr double kSlabExchange = 0.4e-6;
constexpr double kSlabFloor = 4.5e-6;

double unit_seconds(const BatchJobHost &h, bool slab)
{
    const double x = (double)h.job.L / 64.0;
    const double whole = kHalfStepL64 * std::pow(x, kSizeExp);
    const double per_half = slab ? std::max(0.5 * whole + kSlabExchange, kSlabFloor) : whole;
    return 2.0 * (double)std::max<uint64_t>(1, h.job.n_sweeps) * per_half;
}

double simulate_dispatch(const std::vector<std::pair<double, int>> &units, int n_cu)
{
    // units: (cost, 2 for the first workgroup of a pair that starts together, else 1)
    std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
    for (int i = 0; i < n_cu; ++i) free_at.push(0.0);
    double end = 0.0;
    for (size_t i = 0; i < units.size(); ++i) {
        if (units[i].second == 2 && i + 1 < units.size()) {
            const double a = free_at.top();
            free_at.pop();
            const double b = free_at.top();
            free_at.pop();
            const double start = std::max(a, b);
            free_at.push(start + units[i].first);
            free_at.push(start + units[i + 1].first);
            end = std::max(end, start + std::max(units[i].first, units[i + 1].first));
            ++i;
        } else {
            const double a = free_at.top();
            free_at.pop();
            free_at.push(a + units[i].first);
            end = std::max(end, a + units[i].first);
        }
    }
    return end;
}

void choose_split(std::vector<BatchJobHost> &jobs, int n_cu, bool always)
{
    auto splittable = [](const BatchJobHost &h) {
        const TuneCfg d = default_cfg(h.job.L);
        return h.job.L >= ea::kSplitMinL && h.cfg.rw == d.rw && h.cfg.nt == d.nt && h.cfg.sel == ea::SEL_LDS &&
               h.cfg.nt >= 128;
    };
    int best_lmin = 0;
    double best = 0.0;
    for (int lmin : {0, 64, 56, 48}) {
        // every slab must be resident from the start: at most one per CU
        size_t n_slabs = 0;
        for (const BatchJobHost &h : jobs) n_slabs += (lmin && h.job.L >= lmin && splittable(h)) ? 4 : 0;
        if (n_slabs > (size_t)n_cu) continue;
        std::vector<std::pair<double, int>> split, rest;
        for (const BatchJobHost &h : jobs) {
            if (lmin && h.job.L >= lmin && splittable(h)) {
                const double w = unit_seconds(h, true);
                for (int r = 0; r < 2; ++r) {
                    split.push_back({w, 2});
                    split.push_back({w, 1});
                }
            } else {
                const double w = unit_seconds(h, false);
                rest.push_back({w, 1});
                rest.push_back({w, 1});
            }
        }
        std::stable_sort(rest.begin(), rest.end(),
                         [](const std::pair<double, int> &a, const std::pair<double, int> &b) {
                             return a.first > b.first;
                         });
        split.insert(split.end(), rest.begin(), rest.end());
        const double m = simulate_dispatch(split, n_cu);
        if (lmin == 0 || m < best || always) {
            best = m;
            best_lmin = lmin;
        }
    }
    for (BatchJobHost &h : jobs) h.parts = (best_lmin && h.job.L >= best_lmin && splittable(h)) ? 2 : 1;
}

}  // namespace

struct ea_batch {
    std::vector<BatchJobHost> jobs;
    ShellScratch shell_scratch;  // ea_batch_c4_shells
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *buf = nullptr;
    size_t bytes = 0;
    ea::BatchJobDev *d_jobs = nullptr;
    ea::BatchUnit *d_units = nullptr;
    ea::BatchUnit *d_units_graph = nullptr;  // whole-run units read by the captured graph
    uint32_t *d_err = nullptr;                // set by a split pair that gave up waiting
    std::vector<ea::BatchUnit> units;
    size_t lds_bytes = 0;
    std::vector<unsigned long long> h_obs;  // staging for ea_batch_result
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
};


namespace {

ea_status batch_create_cfg(const ea_job *jobs, int32_t n_jobs, void *stream, const TuneCfg *cfgs, int split,
                           ea_batch **out);

// ---------------------------------------------------------------------------
// Autotuner.  For one lattice size it times every valid combination of row
// packing (the default and the next finer one, if its lattice fits LDS),
// working threads per workgroup (256, 512, 768, 1024, capped by the word count)
// and threshold-select variant on a probe batch of 64 samples, keeps only
// candidates whose results equal the default configuration's bit for bit,
// and picks the fastest.  Choices are cached per process and, if the
// environment variable EA_TUNE_CACHE names a file, across processes.

struct TuneRecord {
    TuneCfg cfg;
    double ms = 0.0;
    bool parity_ok = false;
};

std::mutex g_tune_mu;
std::map<int, TuneCfg> g_tuned;
bool g_tune_file_read = false;

std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// Lines "<arch> batch <L> <rw> <nt> <sel> <ms>" of the tuning cache.
void read_tune_file()
{
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char *path = std::getenv("EA_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    const std::string arch = device_arch();
    char line[256], a[64], tag[16];
    int L, rw, nt, sel;
    while (std::fgets(line, sizeof line, f)) {
        if (std::sscanf(line, "%63s %15s %d %d %d %d", a, tag, &L, &rw, &nt, &sel) != 6) continue;
        if (arch != a || std::string(tag) != "batch") continue;
        TuneCfg c;
        c.rw = rw;
        c.nt = nt;
        c.sel = sel;
        if (batch_L_ok(L) && cfg_valid(L, c)) g_tuned[L] = c;
    }
    std::fclose(f);
}

void append_tune_file(int L, const TuneCfg &c, double ms)
{
    const char *path = std::getenv("EA_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s batch %d %d %d %d %.4f\n", device_arch().c_str(), L, c.rw, c.nt, c.sel, ms);
    std::fclose(f);
}

std::vector<TuneCfg> tune_candidates(int L, size_t lds_limit)
{
    std::vector<TuneCfg> out;
    const int R = L / 2, rw0 = ea::words_per_row_c(R), rw1 = ea::finer_words_per_row_c(R, rw0);
    const TuneCfg def = default_cfg(L);
    out.push_back(def);  // the reference comes first
    for (int rw : {rw0, rw1}) {
        if (rw == 0) continue;
        if (4 * (size_t)batch_lds_words(L, rw) + 4 * (size_t)ea::kSelectTableWords > lds_limit) continue;
        const int words = L * L * rw;
        for (int nt : {256, 512, 768, 1024}) {  // 768: three z-planes per thread at L = 48
            if (nt > round_up64(words) && nt != 256) continue;
            for (int sel : {(int)ea::SEL_LDS, (int)ea::SEL_REG}) {
                TuneCfg c;
                c.rw = rw;
                c.nt = std::min(nt, round_up64(words));
                c.sel = sel;
                if (!cfg_valid(L, c)) continue;
                bool dup = false;
                for (const TuneCfg &o : out) dup = dup || (o.rw == c.rw && o.nt == c.nt && o.sel == c.sel);
                if (!dup) out.push_back(c);
            }
        }
    }
    return out;
}

// Run the probe batch with one configuration; returns its results (all
// measurement counters and the final spins, canonical order) and time.
ea_status tune_probe(int L, const TuneCfg &cfg, std::vector<long long> &results, double &ms)
{
    const int n = 64;
    const uint64_t N = (uint64_t)L * L * L;
    const uint64_t sweeps = std::max<uint64_t>(8, (1ull << 22) / N);
    std::vector<uint64_t> meas = {sweeps / 2, sweeps}, tw = {sweeps / 4};
    std::vector<ea_job> jobs((size_t)n);
    for (int i = 0; i < n; ++i) {
        ea_job &j = jobs[(size_t)i];
        j.L = L;
        j.p = (i % 3 == 0) ? 0.2 : 0.5;
        j.T = (i % 2 == 0) ? 0.6 : 1.0;
        j.seed = 1000 + (uint64_t)i;
        j.sample = 0;
        j.n_sweeps = sweeps;
        j.meas_t = meas.data();
        j.n_meas = (int32_t)meas.size();
        j.tw = tw.data();
        j.n_tw = (int32_t)tw.size();
    }
    std::vector<TuneCfg> cfgs((size_t)n, cfg);
    ea_batch *b = nullptr;
    ea_status st = batch_create_cfg(jobs.data(), n, nullptr, cfgs.data(), 1, &b);
    if (st != EA_OK) return st;
    st = ea_batch_run(b, sweeps);  // warm-up
    if (st == EA_OK) st = ea_batch_reset(b);
    if (st == EA_OK) {
        const auto t0 = std::chrono::steady_clock::now();
        st = ea_batch_run(b, sweeps);
        ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    results.clear();
    for (int i = 0; st == EA_OK && i < n; ++i) {
        const BatchJobHost &h = b->jobs[(size_t)i];
        std::vector<unsigned long long> obs((size_t)h.job.n_meas * (size_t)h.obs_stride);
        hipError_t e = hipMemcpy(obs.data(), h.base + h.off_obs, 8 * obs.size(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) st = fail(EA_ERR_DEVICE, "hipMemcpy: %s", hipGetErrorString(e));
        for (unsigned long long v : obs) results.push_back((long long)v);
        if (i < 4) {
            std::vector<int8_t> spins(N);
            for (int r = 0; st == EA_OK && r < 2; ++r) {
                st = read_job_spins(h, r, spins.data(), b->stream);
                for (int8_t v : spins) results.push_back(v);
            }
        }
    }
    ea_batch_destroy(b);
    return st;
}

ea_status tune_lattice(int L, std::vector<TuneRecord> &tried, TuneCfg *best)
{
    int dev = 0, lds_limit = 0;
    EA_HIP(hipGetDevice(&dev));
    EA_HIP(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const std::vector<TuneCfg> cands = tune_candidates(L, (size_t)lds_limit);
    std::vector<long long> ref;
    tried.clear();
    double best_ms = 0.0;
    *best = cands[0];
    for (size_t i = 0; i < cands.size(); ++i) {
        TuneRecord rec;
        rec.cfg = cands[i];
        std::vector<long long> res;
        ea_status st = tune_probe(L, cands[i], res, rec.ms);
        if (st != EA_OK) return st;
        if (i == 0) ref = res;
        rec.parity_ok = res == ref;
        tried.push_back(rec);
        if (rec.parity_ok && (i == 0 || rec.ms < best_ms)) {
            best_ms = rec.ms;
            *best = cands[i];
        }
    }
    return EA_OK;
}

// The configuration a job of size L runs with when tuning is requested.
ea_status tuned_cfg(int L, TuneCfg *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    read_tune_file();
    auto it = g_tuned.find(L);
    if (it != g_tuned.end()) {
        *out = it->second;
        return EA_OK;
    }
    std::vector<TuneRecord> tried;
    TuneCfg best;
    ea_status st = tune_lattice(L, tried, &best);
    if (st != EA_OK) return st;
    g_tuned[L] = best;
    double ms = 0.0;
    for (const TuneRecord &r : tried)
        if (r.cfg.rw == best.rw && r.cfg.nt == best.nt && r.cfg.sel == best.sel) ms = r.ms;
    append_tune_file(L, best, ms);
    *out = best;
    return EA_OK;
}

}  // namespace

namespace {

ea_status batch_create_cfg(const ea_job *jobs, int32_t n_jobs, void *stream, const TuneCfg *cfgs, int split,
                           ea_batch **out)
{
    if (!out) return fail(EA_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!jobs || n_jobs <= 0) return fail(EA_ERR_ARG, "need at least one job");
    ea_batch *b = new (std::nothrow) ea_batch();
    if (!b) return fail(EA_ERR_NOMEM, "host allocation failed");
    b->jobs.resize((size_t)n_jobs);
    size_t off = 0;
    int max_lds = 0;
    std::vector<size_t> region((size_t)n_jobs);
    for (int32_t j = 0; j < n_jobs; ++j) {
        ea_status st = plan_job(jobs[j], j, b->jobs[(size_t)j], cfgs ? &cfgs[j] : nullptr);
        if (st != EA_OK) {
            delete b;
            return st;
        }
        region[(size_t)j] = off = align256(off);
        off += b->jobs[(size_t)j].bytes;
    }
    if (split != 1) {
        int dev = 0, n_cu = 0;
        hipError_t e0 = hipGetDevice(&dev);
        if (e0 == hipSuccess) e0 = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e0 != hipSuccess) {
            delete b;
            return fail(EA_ERR_DEVICE, "device query: %s", hipGetErrorString(e0));
        }
        choose_split(b->jobs, n_cu, split == 2);
    }
    for (const BatchJobHost &h : b->jobs) max_lds = std::max(max_lds, job_lds_words(h));
    const size_t off_jobs = align256(off);
    off = off_jobs + sizeof(ea::BatchJobDev) * (size_t)n_jobs;
    const size_t off_units = align256(off);
    off = off_units + sizeof(ea::BatchUnit) * 4 * (size_t)n_jobs;
    const size_t off_units_graph = align256(off);
    off = off_units_graph + sizeof(ea::BatchUnit) * 4 * (size_t)n_jobs;
    const size_t off_err = align256(off);
    off = off_err + 4;
    b->bytes = align256(off);
    b->lds_bytes = (size_t)max_lds * 4;  // dynamic part; the select tables are static

    ea_status st = prepare_batch_lds(b->lds_bytes);
    if (st != EA_OK) {
        delete b;
        return st;
    }
    hipError_t e;
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else {
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete b;
            return fail(EA_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        b->own_stream = true;
    }
    e = hipMalloc((void **)&b->buf, b->bytes);
    if (e != hipSuccess) {
        ea_batch_destroy(b);
        return fail(EA_ERR_NOMEM, "hipMalloc(%zu): %s", b->bytes, hipGetErrorString(e));
    }
    std::vector<ea::BatchJobDev> dj((size_t)n_jobs);
    std::vector<BatchJobHost *> ptrs;
    std::vector<uint64_t> span;
    b->d_err = (uint32_t *)(b->buf + off_err);
    for (int32_t j = 0; j < n_jobs; ++j) {
        BatchJobHost &h = b->jobs[(size_t)j];
        h.base = b->buf + region[(size_t)j];
        h.err = b->d_err;
        dj[(size_t)j] = make_job_dev(h);
        st = upload_schedule(h, b->stream);
        if (st != EA_OK) {
            ea_batch_destroy(b);
            return st;
        }
        ptrs.push_back(&h);
        span.push_back(h.job.n_sweeps);
    }
    b->d_jobs = (ea::BatchJobDev *)(b->buf + off_jobs);
    b->d_units = (ea::BatchUnit *)(b->buf + off_units);
    b->d_units_graph = (ea::BatchUnit *)(b->buf + off_units_graph);
    e = hipMemcpyAsync(b->d_jobs, dj.data(), sizeof(ea::BatchJobDev) * dj.size(), hipMemcpyHostToDevice,
                       b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        ea_batch_destroy(b);
        return fail(EA_ERR_DEVICE, "job table upload: %s", hipGetErrorString(e));
    }
    order_units(ptrs, span, b->units);
    st = ea_batch_reset(b);
    if (st != EA_OK) {
        ea_batch_destroy(b);
        return st;
    }
    *out = b;
    return EA_OK;
}

// Generate every job's initial state and clear the counters (also what a
// captured run starts with).
ea_status reset_batch_device(ea_batch *b)
{
    hipLaunchKernelGGL(ea::zero_u32_kernel, dim3(1), dim3(64), 0, b->stream, b->d_err, (size_t)1);
    EA_HIP(hipGetLastError());
    for (auto &h : b->jobs) {
        ea_status st = init_job_device(h, b->stream);
        if (st != EA_OK) return st;
    }
    return EA_OK;
}

// After a synchronised run: did a split pair give up waiting?
ea_status check_batch_err(ea_batch *b)
{
    uint32_t err = 0;
    EA_HIP(hipMemcpyAsync(&err, b->d_err, 4, hipMemcpyDeviceToHost, b->stream));
    EA_HIP(hipStreamSynchronize(b->stream));
    if (err) return fail(EA_ERR_DEVICE, "the two workgroups of a split replica did not meet; results are invalid");
    return EA_OK;
}

}  // namespace

extern "C" {

ea_status ea_batch_create(const ea_job *jobs, int32_t n_jobs, const ea_batch_opts *opts, ea_batch **out)
{
    if (!out) return fail(EA_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!jobs || n_jobs <= 0) return fail(EA_ERR_ARG, "need at least one job");
    std::vector<TuneCfg> cfgs((size_t)n_jobs);
    for (int32_t j = 0; j < n_jobs; ++j) {
        if (!batch_L_ok(jobs[j].L))
            return fail(EA_ERR_ARG, "job %d: L=%d must be a multiple of 8 in [8, %d] for the batched form", j,
                        jobs[j].L, ea::kBatchMaxL);
        cfgs[(size_t)j] = default_cfg(jobs[j].L);
        if (opts && opts->autotune) {
            ea_status st = tuned_cfg(jobs[j].L, &cfgs[(size_t)j]);
            if (st != EA_OK) return st;
        }
    }
    const int split = opts ? opts->split : 0;
    if (split < 0 || split > 2) return fail(EA_ERR_ARG, "split=%d is not 0, 1 or 2", split);
    return batch_create_cfg(jobs, n_jobs, opts ? opts->stream : nullptr, cfgs.data(), split, out);
}

ea_status ea_tune(int32_t L, int32_t force, ea_tune_choice *chosen, ea_tune_choice *tried, int32_t max_tried,
                  int32_t *n_tried)
{
    if (!chosen) return fail(EA_ERR_ARG, "chosen is NULL");
    if (!batch_L_ok(L)) return fail(EA_ERR_ARG, "L=%d has no batched configuration", L);
    std::vector<TuneRecord> recs;
    TuneCfg best;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        read_tune_file();
        auto it = g_tuned.find(L);
        if (it != g_tuned.end() && !force) {
            best = it->second;
        } else {
            ea_status st = tune_lattice(L, recs, &best);
            if (st != EA_OK) return st;
            g_tuned[L] = best;
            double ms = 0.0;
            for (const TuneRecord &r : recs)
                if (r.cfg.rw == best.rw && r.cfg.nt == best.nt && r.cfg.sel == best.sel) ms = r.ms;
            append_tune_file(L, best, ms);
        }
    }
    auto put = [](ea_tune_choice *c, const TuneCfg &cfg, double ms, bool ok) {
        c->words_per_row = cfg.rw;
        c->threads = cfg.nt;
        c->select = cfg.sel;
        c->ms = ms;
        c->parity_ok = ok ? 1 : 0;
    };
    double best_ms = 0.0;
    for (const TuneRecord &r : recs)
        if (r.cfg.rw == best.rw && r.cfg.nt == best.nt && r.cfg.sel == best.sel) best_ms = r.ms;
    put(chosen, best, best_ms, true);
    if (n_tried) *n_tried = (int32_t)recs.size();
    for (size_t i = 0; tried && i < recs.size() && (int32_t)i < max_tried; ++i)
        put(&tried[i], recs[i].cfg, recs[i].ms, recs[i].parity_ok);
    return EA_OK;
}

void ea_batch_destroy(ea_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->buf) (void)hipFree(b->buf);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

ea_status ea_batch_reset(ea_batch *b)
{
    if (!b) return fail(EA_ERR_ARG, "batch is NULL");
    return reset_batch_device(b);
}

ea_status ea_batch_run(ea_batch *b, uint64_t t_stop)
{
    if (!b) return fail(EA_ERR_ARG, "batch is NULL");
    bool any = false;
    for (auto &u : b->units) {
        const BatchJobHost &h = b->jobs[(size_t)u.job];
        const uint64_t stop = std::min<uint64_t>(t_stop, h.job.n_sweeps);
        u.t_stop = (uint32_t)std::max<uint64_t>(stop, h.t_host);
        u.first = h.started ? 0 : 1;
        any = any || u.t_stop > h.t_host || u.first;
    }
    if (!any) return EA_OK;
    std::vector<ea::BatchUnit> launch = b->units;
    debug_order_units(b->jobs.data(), launch);
    EA_HIP(hipMemcpyAsync(b->d_units, launch.data(), sizeof(ea::BatchUnit) * launch.size(),
                          hipMemcpyHostToDevice, b->stream));
    hipLaunchKernelGGL(ea::batch_kernel, dim3((unsigned)launch.size()), dim3(ea::kBatchThreads), b->lds_bytes,
                       b->stream, b->d_jobs, b->d_units, debug_poison_word(), (int)(b->lds_bytes / 4));
    EA_HIP(hipGetLastError());
    for (auto &h : b->jobs) {
        h.t_host = std::max<uint64_t>(h.t_host, std::min<uint64_t>(t_stop, h.job.n_sweeps));
        h.started = true;
    }
    // the unit table is read by the kernel: keep the host copy stable until it ran
    EA_HIP(hipStreamSynchronize(b->stream));
    return check_batch_err(b);
}

ea_status ea_batch_capture(ea_batch *b)
{
    if (!b) return fail(EA_ERR_ARG, "batch is NULL");
    if (b->graph_exec) return EA_OK;
    // the whole-run unit table goes to the device once, outside the graph
    std::vector<ea::BatchUnit> full = b->units;
    for (auto &u : full) {
        u.t_stop = (uint32_t)b->jobs[(size_t)u.job].job.n_sweeps;
        u.first = 1;
    }
    debug_order_units(b->jobs.data(), full);
    EA_HIP(hipMemcpyAsync(b->d_units_graph, full.data(), sizeof(ea::BatchUnit) * full.size(),
                          hipMemcpyHostToDevice, b->stream));
    EA_HIP(hipStreamSynchronize(b->stream));
    EA_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    ea_status st = reset_batch_device(b);
    if (st == EA_OK)
        hipLaunchKernelGGL(ea::batch_kernel, dim3((unsigned)full.size()), dim3(ea::kBatchThreads), b->lds_bytes,
                           b->stream, b->d_jobs, b->d_units_graph, debug_poison_word(), (int)(b->lds_bytes / 4));
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (st != EA_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(EA_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph_exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(EA_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    b->graph = graph;
    return EA_OK;
}

ea_status ea_batch_replay(ea_batch *b)
{
    if (!b) return fail(EA_ERR_ARG, "batch is NULL");
    if (!b->graph_exec) return fail(EA_ERR_STATE, "ea_batch_capture first");
    EA_HIP(hipGraphLaunch(b->graph_exec, b->stream));
    EA_HIP(hipStreamSynchronize(b->stream));
    for (auto &h : b->jobs) {
        h.t_host = h.job.n_sweeps;
        h.started = true;
    }
    return check_batch_err(b);
}

ea_status ea_batch_time(ea_batch *b, int32_t job, uint64_t *t)
{
    if (!b || !t) return fail(EA_ERR_ARG, "NULL argument");
    if (job < 0 || job >= (int32_t)b->jobs.size()) return fail(EA_ERR_ARG, "job %d out of range", job);
    *t = b->jobs[(size_t)job].t_host;
    return EA_OK;
}

ea_status ea_batch_result(ea_batch *b, int32_t job, int32_t k, ea_obs *out)
{
    if (!b || !out) return fail(EA_ERR_ARG, "NULL argument");
    if (job < 0 || job >= (int32_t)b->jobs.size()) return fail(EA_ERR_ARG, "job %d out of range", job);
    const BatchJobHost &h = b->jobs[(size_t)job];
    if (k < 0 || k >= h.job.n_meas) return fail(EA_ERR_ARG, "measurement %d out of range", k);
    if (h.meas_t[(size_t)k] > h.t_host || !h.started)
        return fail(EA_ERR_STATE, "measurement %d (t=%u) not reached", k, h.meas_t[(size_t)k]);
    b->h_obs.resize((size_t)h.obs_stride);
    EA_HIP(hipMemcpyAsync(b->h_obs.data(), h.base + h.off_obs + 8 * (size_t)k * (size_t)h.obs_stride,
                          8 * (size_t)h.obs_stride, hipMemcpyDeviceToHost, b->stream));
    EA_HIP(hipStreamSynchronize(b->stream));
    return fill_obs(h, b->h_obs.data(), k, out);
}

ea_status ea_batch_parts(ea_batch *b, int32_t job, int32_t *parts)
{
    if (!b || !parts) return fail(EA_ERR_ARG, "NULL argument");
    if (job < 0 || job >= (int32_t)b->jobs.size()) return fail(EA_ERR_ARG, "job %d out of range", job);
    *parts = b->jobs[(size_t)job].parts;
    return EA_OK;
}

ea_status ea_batch_get_spins(ea_batch *b, int32_t job, int32_t r, int8_t *pm1)
{
    if (!b || !pm1) return fail(EA_ERR_ARG, "NULL argument");
    if (job < 0 || job >= (int32_t)b->jobs.size()) return fail(EA_ERR_ARG, "job %d out of range", job);
    if (r < 0 || r > 1) return fail(EA_ERR_ARG, "replica %d not 0 or 1", r);
    return read_job_spins(b->jobs[(size_t)job], r, pm1, b->stream);
}

}  // extern "C"
