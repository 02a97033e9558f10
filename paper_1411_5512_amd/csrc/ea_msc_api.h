// ea_msc_api.h -- host side of the multispin-coded batch (asynchronous
// multispin coding, Sec. III).  Included by ea_api.hip after its helpers.
#pragma once

#include "ea_msc_kernels.h"

struct ea_msc {
    ShellScratch shell_scratch;  // ea_msc_c4_shells
    int L = 0, B = 0, M = 0, S = 0, G = 0;
    ea::MscGeom geom{};
    double p = 0, T = 0;
    uint64_t seed = 0;
    uint32_t sample0 = 0, shared = 0;
    uint32_t thr[3] = {0, 0, 0};
    uint64_t pcut = 0;
    uint64_t t = 0;
    int n_slots = 0;
    std::vector<uint64_t> snap_t;
    std::vector<char> snap_taken;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *buf = nullptr;
    bool own_buf = false;
    ea::MscLattice lat{};
    uint32_t *snaps = nullptr;
    unsigned long long *meas = nullptr;
    uint32_t *t_dev = nullptr;
    uint32_t *q = nullptr;  // overlap words for the C4 passes
    size_t spin_words = 0, bond_words = 0, n_count = 0;
    std::vector<unsigned long long> host_meas;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    uint32_t graph_order = 0;  // debug order the graph was captured with
};

namespace {

#define EA_DISPATCH_M(M, ...)                                                           \
    do {                                                                                \
        switch (M) {                                                                    \
        case 1: { constexpr int MM = 1; __VA_ARGS__; } break;                           \
        case 2: { constexpr int MM = 2; __VA_ARGS__; } break;                           \
        case 4: { constexpr int MM = 4; __VA_ARGS__; } break;                           \
        case 8: { constexpr int MM = 8; __VA_ARGS__; } break;                           \
        case 16: { constexpr int MM = 16; __VA_ARGS__; } break;                         \
        default: { constexpr int MM = 32; __VA_ARGS__; } break;                         \
        }                                                                               \
    } while (0)

uint32_t key_lo_u64(uint64_t seed) { return (uint32_t)(seed & 0xffffffffu); }
uint32_t key_hi_u64(uint64_t seed) { return (uint32_t)(seed >> 32); }

constexpr int kMscMaxSamples = 256;  // eight word sets
constexpr int kMscQuantities = ea::MSC_AUTO + 2 * kMaxSlots;  // counters before the C4 block

struct MscLayout {
    int L, B, M, S, G, Lz, R, P;
    size_t spin_words, bond_words, snap_words, n_count;
    size_t off_spins, off_bonds, off_snaps, off_q, off_meas, off_ctl, total;
};

ea_status msc_layout(const ea_msc_config *cfg, MscLayout &y)
{
    if (!cfg) return fail(EA_ERR_ARG, "config is NULL");
    if (!valid_L(cfg->L)) return fail(EA_ERR_ARG, "L=%d must be a multiple of 8 in [8, %d]", cfg->L, kMaxL);
    const int B = cfg->n_samples;
    if (!(B == 1 || B == 2 || B == 4 || B == 8 || B == 16 || (B % 32 == 0 && B >= 32 && B <= kMscMaxSamples)))
        return fail(EA_ERR_ARG, "n_samples=%d is not 1, 2, 4, 8, 16 or a multiple of 32 up to %d", B,
                    kMscMaxSamples);
    y.L = cfg->L;
    y.B = B;
    y.M = B < 32 ? B : 32;
    y.S = 32 / y.M;
    y.G = B / y.M;
    if (y.L % (2 * y.S) != 0)
        return fail(EA_ERR_ARG, "n_samples=%d cuts L=%d into %d slabs, which needs L divisible by %d", B, y.L, y.S,
                    2 * y.S);
    if (cfg->n_tw_slots < 0 || cfg->n_tw_slots > kMaxSlots)
        return fail(EA_ERR_ARG, "n_tw_slots=%d outside [0, %d]", cfg->n_tw_slots, kMaxSlots);
    y.Lz = y.L / y.S;
    y.R = y.L / 2;
    y.P = y.R * y.L * y.Lz;
    y.spin_words = (size_t)y.G * 4 * (size_t)y.P;
    y.bond_words = (size_t)y.G * 6 * (size_t)y.P;
    y.snap_words = (size_t)cfg->n_tw_slots * y.spin_words;
    y.n_count = ((size_t)kMscQuantities + 3 * (size_t)(y.R + 1)) * (size_t)y.G * 32;
    y.off_spins = 0;
    y.off_bonds = align256(y.off_spins + 4 * y.spin_words);
    y.off_snaps = align256(y.off_bonds + 4 * y.bond_words);
    y.off_q = align256(y.off_snaps + 4 * y.snap_words);
    y.off_meas = align256(y.off_q + 4 * (y.spin_words / 2));
    y.off_ctl = align256(y.off_meas + 8 * y.n_count);
    y.total = align256(y.off_ctl + 256);
    return EA_OK;
}

ea_status msc_half_step(ea_msc *s, int half, uint32_t t_off)
{
    ea::MscGeom g = s->geom;
    g.order = debug_grid_order();
    // two blocks (one per replica) per tile of 256 threads; grid.y = word set
    const dim3 grid(2 * blocks_for((size_t)g.q), (unsigned)s->G, 1);
    EA_DISPATCH_M(s->M, hipLaunchKernelGGL((ea::msc_half_step_kernel<MM>), grid, dim3(256), 0, s->stream, s->lat,
                                            g, half, s->t_dev, t_off, key_lo_u64(s->seed), key_hi_u64(s->seed),
                                            s->shared, s->thr[0], s->thr[1], s->thr[2]));
    return EA_OK;
}

ea_status msc_sweeps(ea_msc *s, uint32_t n)
{
    for (uint32_t i = 0; i < n; ++i) {
        msc_half_step(s, 0, i);
        msc_half_step(s, 1, i);
    }
    return EA_OK;
}

ea_status msc_build_graph(ea_msc *s)
{
    s->graph_order = debug_grid_order();
    EA_HIP(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    ea_status st = msc_sweeps(s, kGraphSweeps);
    hipLaunchKernelGGL(ea::advance_u32_kernel, dim3(1), dim3(64), 0, s->stream, s->t_dev, kGraphSweeps);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s->stream, &graph);
    if (st != EA_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(EA_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&s->graph_exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(EA_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    s->graph = graph;
    return EA_OK;
}

// Bit of sample b at canonical site (x, y, z) in a word set's plane pair:
// word index within colour c's plane and bit position.
struct MscBit {
    int gi, c;
    size_t hw;
    int bit;
};

MscBit msc_bit(const ea_msc *s, int b, int x, int y, int z)
{
    MscBit r;
    const int m = b % s->M, k = z / s->geom.Lz, zr = z - k * s->geom.Lz;
    r.gi = b / s->M;
    r.c = (x + y + z) & 1;
    r.hw = (size_t)(x >> 1) + (size_t)s->geom.R * ((size_t)y + (size_t)s->L * (size_t)zr);
    r.bit = k * s->M + m;
    return r;
}

ea_status msc_check_sample(const ea_msc *s, int32_t b)
{
    if (!s) return fail(EA_ERR_ARG, "batch is NULL");
    if (b < 0 || b >= s->B) return fail(EA_ERR_ARG, "sample %d outside [0, %d)", b, s->B);
    return EA_OK;
}

}  // namespace

ea_status ea_msc_footprint(const ea_msc_config *cfg, size_t *bytes)
{
    if (!bytes) return fail(EA_ERR_ARG, "NULL argument");
    MscLayout y{};
    ea_status st = msc_layout(cfg, y);
    if (st != EA_OK) return st;
    *bytes = y.total;
    return EA_OK;
}

void ea_msc_destroy(ea_msc *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->own_buf && s->buf) (void)hipFree(s->buf);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

ea_status ea_msc_create(const ea_msc_config *cfg, ea_msc **out)
{
    if (!cfg || !out) return fail(EA_ERR_ARG, "NULL argument");
    *out = nullptr;
    MscLayout y{};
    ea_status st = msc_layout(cfg, y);
    if (st != EA_OK) return st;
    if (!(cfg->p >= 0.0 && cfg->p <= 1.0)) return fail(EA_ERR_ARG, "p=%g outside [0, 1]", cfg->p);
    if (!(cfg->T >= 0.0) || !std::isfinite(cfg->T)) return fail(EA_ERR_ARG, "T=%g must be finite and >= 0", cfg->T);
    if (cfg->dev_buf) {
        if (cfg->dev_buf_bytes < y.total)
            return fail(EA_ERR_ARG, "dev_buf holds %zu bytes, %zu needed", cfg->dev_buf_bytes, y.total);
        if (((uintptr_t)cfg->dev_buf & 255) != 0) return fail(EA_ERR_ARG, "dev_buf is not 256-byte aligned");
    }
    ea_msc *s = new (std::nothrow) ea_msc();
    if (!s) return fail(EA_ERR_NOMEM, "host allocation failed");
    s->L = y.L;
    s->B = y.B;
    s->M = y.M;
    s->S = y.S;
    s->G = y.G;
    s->geom.L = y.L;
    s->geom.R = y.R;
    s->geom.Lz = y.Lz;
    s->geom.P = y.P;
    s->geom.q = y.P / 4;
    s->geom.by_r4.m = ((uint64_t)1 << 40) / (uint64_t)(y.R / 4) + 1;
    s->geom.by_l.m = ((uint64_t)1 << 40) / (uint64_t)y.L + 1;
    s->p = cfg->p;
    s->T = cfg->T;
    s->seed = cfg->seed;
    s->sample0 = cfg->sample0;
    s->shared = cfg->shared;
    s->n_slots = cfg->n_tw_slots;
    s->snap_t.assign((size_t)s->n_slots, 0);
    s->snap_taken.assign((size_t)s->n_slots, 0);
    s->spin_words = y.spin_words;
    s->bond_words = y.bond_words;
    s->n_count = y.n_count;
    s->host_meas.assign(y.n_count, 0);
    host_thresholds(cfg->T, s->thr);
    s->pcut = (uint64_t)std::floor(std::ldexp(cfg->p, 32));

    hipError_t e;
    if (cfg->stream) {
        s->stream = (hipStream_t)cfg->stream;
    } else {
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete s;
            return fail(EA_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        s->own_stream = true;
    }
    if (cfg->dev_buf) {
        s->buf = (char *)cfg->dev_buf;
    } else {
        e = hipMalloc((void **)&s->buf, y.total);
        if (e != hipSuccess) {
            ea_msc_destroy(s);
            return fail(EA_ERR_NOMEM, "hipMalloc(%zu): %s", y.total, hipGetErrorString(e));
        }
        s->own_buf = true;
    }
    s->lat.spins = (uint32_t *)(s->buf + y.off_spins);
    s->lat.bonds = (uint32_t *)(s->buf + y.off_bonds);
    s->snaps = (uint32_t *)(s->buf + y.off_snaps);
    s->meas = (unsigned long long *)(s->buf + y.off_meas);
    s->q = (uint32_t *)(s->buf + y.off_q);
    s->t_dev = (uint32_t *)(s->buf + y.off_ctl);

    const dim3 grid(blocks_for((size_t)s->geom.q), 5, 2 * (unsigned)s->G);
    EA_DISPATCH_M(s->M, hipLaunchKernelGGL((ea::msc_init_kernel<MM>), grid, dim3(256), 0, s->stream, s->lat,
                                            s->geom, key_lo_u64(s->seed), key_hi_u64(s->seed), s->sample0, s->pcut));
    if (y.snap_words) {
        hipLaunchKernelGGL(ea::zero_u32_kernel, dim3(blocks_for(y.snap_words)), dim3(256), 0, s->stream, s->snaps,
                           y.snap_words);
    }
    e = hipGetLastError();
    if (e != hipSuccess) {
        ea_msc_destroy(s);
        return fail(EA_ERR_DEVICE, "initial state: %s", hipGetErrorString(e));
    }
    *out = s;
    return EA_OK;
}

ea_status ea_msc_sweep(ea_msc *s, uint64_t n)
{
    if (!s) return fail(EA_ERR_ARG, "batch is NULL");
    if (s->t + n >= (1ull << 32) || n >= (1ull << 32))
        return fail(EA_ERR_ARG, "t + n = %llu would reach 2^32", (unsigned long long)(s->t + n));
    if (n == 0) return EA_OK;
    hipLaunchKernelGGL(ea::set_u32_kernel, dim3(1), dim3(64), 0, s->stream, s->t_dev, (uint32_t)s->t);
    uint64_t left = n;
    if (left >= kGraphSweeps) {
        if (s->graph_exec && s->graph_order != debug_grid_order()) {
            // captured under another debug order: capture again
            (void)hipGraphExecDestroy(s->graph_exec);
            (void)hipGraphDestroy(s->graph);
            s->graph_exec = nullptr;
            s->graph = nullptr;
        }
        if (!s->graph_exec) {
            ea_status st = msc_build_graph(s);
            if (st != EA_OK) return st;
        }
        // each replay advances the device counter by kGraphSweeps
        for (; left >= kGraphSweeps; left -= kGraphSweeps) EA_HIP(hipGraphLaunch(s->graph_exec, s->stream));
    }
    msc_sweeps(s, (uint32_t)left);
    EA_HIP(hipGetLastError());
    s->t += n;
    return EA_OK;
}

ea_status ea_msc_snapshot(ea_msc *s, int32_t slot)
{
    if (!s) return fail(EA_ERR_ARG, "batch is NULL");
    if (slot < 0 || slot >= s->n_slots) return fail(EA_ERR_ARG, "slot %d outside [0, %d)", slot, s->n_slots);
    hipLaunchKernelGGL(ea::copy_words_kernel, dim3(blocks_for(s->spin_words)), dim3(256), 0, s->stream,
                       s->snaps + (size_t)slot * s->spin_words, s->lat.spins, s->spin_words);
    EA_HIP(hipGetLastError());
    s->snap_t[(size_t)slot] = s->t;
    s->snap_taken[(size_t)slot] = 1;
    return EA_OK;
}

ea_status ea_msc_measure(ea_msc *s, ea_obs *out)
{
    if (!s || !out) return fail(EA_ERR_ARG, "NULL argument");
    const ea::MscGeom g = s->geom;
    bool any_auto = false, any_c4 = false;
    for (int b = 0; b < s->B; ++b) {
        if (out[b].autocorr && out[b].n_tw != s->n_slots)
            return fail(EA_ERR_ARG, "sample %d: n_tw=%d but the batch has %d slots", b, out[b].n_tw, s->n_slots);
        if (out[b].c4 && out[b].rmax != g.R)
            return fail(EA_ERR_ARG, "sample %d: rmax=%d but L/2=%d", b, out[b].rmax, g.R);
        any_auto = any_auto || (out[b].autocorr && s->n_slots > 0);
        any_c4 = any_c4 || out[b].c4;
    }
    hipLaunchKernelGGL(ea::zero_u64_kernel, dim3(blocks_for(s->n_count)), dim3(256), 0, s->stream, s->meas,
                       s->n_count);
    const unsigned nblk = (unsigned)std::min<size_t>(blocks_for(2 * (size_t)g.P), 512);
    const dim3 grid(nblk, 1 + (any_auto ? (unsigned)s->n_slots : 0u), (unsigned)s->G);
    EA_DISPATCH_M(s->M, hipLaunchKernelGGL((ea::msc_measure_kernel<MM>), grid, dim3(256), 0, s->stream, s->lat, g,
                                            s->snaps, s->spin_words, s->G, s->meas));
    unsigned long long *c4_acc = s->meas + (size_t)kMscQuantities * s->G * 32;
    if (any_c4) {
        hipLaunchKernelGGL(ea::msc_q_kernel, dim3(blocks_for(s->spin_words / 2)), dim3(256), 0, s->stream, s->lat, g,
                           s->G, s->q);
        const unsigned nblk_c4 = (unsigned)std::min<size_t>(blocks_for(2 * (size_t)g.P), 64);
        const dim3 grid_c4(nblk_c4, (unsigned)(g.R + 1), (unsigned)s->G);
        const size_t axis = (size_t)(g.R + 1) * s->G * 32;  // counters of one axis
        EA_DISPATCH_M(s->M, hipLaunchKernelGGL((ea::msc_c4_kernel<MM, 0>), grid_c4, dim3(256), 0, s->stream, s->q,
                                                g, s->G, c4_acc));
        EA_DISPATCH_M(s->M, hipLaunchKernelGGL((ea::msc_c4_kernel<MM, 1>), grid_c4, dim3(256), 0, s->stream, s->q,
                                                g, s->G, c4_acc + axis));
        EA_DISPATCH_M(s->M, hipLaunchKernelGGL((ea::msc_c4_kernel<MM, 2>), grid_c4, dim3(256), 0, s->stream, s->q,
                                                g, s->G, c4_acc + 2 * axis));
    }
    EA_HIP(hipGetLastError());
    EA_HIP(hipMemcpyAsync(s->host_meas.data(), s->meas, s->n_count * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));

    const int64_t N = (int64_t)s->L * s->L * s->L;
    const unsigned long long *h = s->host_meas.data();
    for (int b = 0; b < s->B; ++b) {
        const int gi = b / s->M, m = b % s->M;
        // quantity q of sample b: its S bits k M + m
        auto count = [&](size_t q) {
            int64_t v = 0;
            for (int k = 0; k < s->S; ++k) v += (int64_t)h[(q * s->G + gi) * 32 + (size_t)(k * s->M + m)];
            return v;
        };
        ea_obs &o = out[b];
        o.t = s->t;
        for (int r = 0; r < 2; ++r) {
            o.unsat[r] = count(ea::MSC_UNSAT + r);
            o.mag[r] = N - 2 * count(ea::MSC_DOWN + r);
        }
        o.overlap = N - 2 * count(ea::MSC_QDIFF);
        if (o.autocorr) {
            for (int r = 0; r < 2; ++r)
                for (int k = 0; k < s->n_slots; ++k)
                    o.autocorr[r * s->n_slots + k] =
                        s->snap_taken[(size_t)k] ? N - 2 * count(ea::MSC_AUTO + 2 * (size_t)k + r) : 0;
            if (o.tw)
                for (int k = 0; k < s->n_slots; ++k) o.tw[k] = s->snap_t[(size_t)k];
        }
        if (o.c4)
            for (int i = 0; i < 3 * (g.R + 1); ++i) o.c4[i] = N - 2 * count((size_t)kMscQuantities + (size_t)i);
    }
    return EA_OK;
}

ea_status ea_msc_get_spins(ea_msc *s, int32_t b, int32_t r, int8_t *pm1)
{
    ea_status st = msc_check_sample(s, b);
    if (st != EA_OK) return st;
    if (r < 0 || r > 1 || !pm1) return fail(EA_ERR_ARG, "replica %d or NULL output", r);
    const int gi = b / s->M;
    const size_t P = (size_t)s->geom.P;
    std::vector<uint32_t> w(2 * P);
    EA_HIP(hipMemcpyAsync(w.data(), s->lat.spins + ((size_t)gi * 2 + (size_t)r) * 2 * P, 2 * P * 4,
                          hipMemcpyDeviceToHost, s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));
    const int L = s->L;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const MscBit q = msc_bit(s, b, x, y, z);
                const uint32_t v = (w[(size_t)q.c * P + q.hw] >> q.bit) & 1u;
                pm1[(size_t)x + (size_t)L * ((size_t)y + (size_t)L * z)] = v ? -1 : 1;
            }
    return EA_OK;
}

ea_status ea_msc_set_spins(ea_msc *s, int32_t b, int32_t r, const int8_t *pm1)
{
    ea_status st = msc_check_sample(s, b);
    if (st != EA_OK) return st;
    if (r < 0 || r > 1 || !pm1) return fail(EA_ERR_ARG, "replica %d or NULL input", r);
    const int L = s->L;
    const size_t N = (size_t)L * L * L;
    for (size_t i = 0; i < N; ++i)
        if (pm1[i] != 1 && pm1[i] != -1) return fail(EA_ERR_ARG, "spin %zu is %d, not +-1", i, (int)pm1[i]);
    const int gi = b / s->M;
    const size_t P = (size_t)s->geom.P;
    uint32_t *dev = s->lat.spins + ((size_t)gi * 2 + (size_t)r) * 2 * P;
    std::vector<uint32_t> w(2 * P);
    EA_HIP(hipMemcpyAsync(w.data(), dev, 2 * P * 4, hipMemcpyDeviceToHost, s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const MscBit q = msc_bit(s, b, x, y, z);
                uint32_t &word = w[(size_t)q.c * P + q.hw];
                const uint32_t v = pm1[(size_t)x + (size_t)L * ((size_t)y + (size_t)L * z)] < 0 ? 1u : 0u;
                word = (word & ~(1u << q.bit)) | (v << q.bit);
            }
    EA_HIP(hipMemcpyAsync(dev, w.data(), 2 * P * 4, hipMemcpyHostToDevice, s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));
    return EA_OK;
}

ea_status ea_msc_get_bonds(ea_msc *s, int32_t b, int8_t *pm1)
{
    ea_status st = msc_check_sample(s, b);
    if (st != EA_OK) return st;
    if (!pm1) return fail(EA_ERR_ARG, "NULL output");
    const int gi = b / s->M;
    const size_t P = (size_t)s->geom.P;
    std::vector<uint32_t> w(6 * P);
    EA_HIP(hipMemcpyAsync(w.data(), s->lat.bonds + (size_t)gi * 6 * P, 6 * P * 4, hipMemcpyDeviceToHost,
                          s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));
    const int L = s->L;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const MscBit q = msc_bit(s, b, x, y, z);
                const size_t site = (size_t)x + (size_t)L * ((size_t)y + (size_t)L * z);
                for (int d = 0; d < 3; ++d) {
                    const uint32_t v = (w[((size_t)d * 2 + (size_t)q.c) * P + q.hw] >> q.bit) & 1u;
                    pm1[3 * site + (size_t)d] = v ? -1 : 1;
                }
            }
    return EA_OK;
}

ea_status ea_msc_time(const ea_msc *s, uint64_t *t)
{
    if (!s || !t) return fail(EA_ERR_ARG, "NULL argument");
    *t = s->t;
    return EA_OK;
}

ea_status ea_msc_set_time(ea_msc *s, uint64_t t)
{
    if (!s) return fail(EA_ERR_ARG, "batch is NULL");
    if (t >= (1ull << 32)) return fail(EA_ERR_ARG, "t=%llu must be below 2^32", (unsigned long long)t);
    s->t = t;
    return EA_OK;
}

ea_status ea_msc_sync(ea_msc *s)
{
    if (!s) return fail(EA_ERR_ARG, "batch is NULL");
    EA_HIP(hipStreamSynchronize(s->stream));
    return EA_OK;
}
