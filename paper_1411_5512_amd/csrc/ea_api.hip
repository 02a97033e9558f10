// ea_api.hip -- host side of the C ABI declared in include/ea.h: argument
// checks, device memory, layout conversion and kernel dispatch for the plain
// form (one launch per checkerboard half-step).
#include "ea.h"
#include "ea_batch_kernels.h"
#include "ea_slab_kernels.h"
#include "ea_shells.h"
#include "ea_fft.h"

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace {

thread_local std::string g_last_error;

ea_status fail(ea_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define EA_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(EA_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr int kMaxSlots = 64;
constexpr int kMaxL = 256;

// Race and order debug mode (ea_set_debug): read at every launch.
std::atomic<uint32_t> g_debug_flags{0}, g_debug_seed{0};

// Order word of the grid launches (ea::debug_block): bit 31 reverses, bits
// 0..30 rotate; 0 = the default order.
uint32_t debug_grid_order()
{
    const uint32_t f = g_debug_flags.load();
    uint32_t o = 0;
    if (f & EA_DEBUG_REVERSE) o |= 0x80000000u;
    if (f & EA_DEBUG_ROTATE) o |= g_debug_seed.load() & 0x7fffffffu;
    return o;
}

// LDS fill pattern of the persistent kernels (ea::debug_poison); 0 = off.
uint32_t debug_poison_word()
{
    if (!(g_debug_flags.load() & EA_DEBUG_POISON)) return 0;
    const uint32_t w = 0xA5C3E187u ^ (g_debug_seed.load() * 0x9E3779B9u);
    return w ? w : 0xFFFFFFFFu;
}

// The same order on the host, for lists of units: position i of the list
// run by workgroup i becomes position perm(i).
template <class T>
void debug_permute(T *v, size_t n)
{
    const uint32_t o = debug_grid_order();
    if (o == 0 || n < 2) return;
    std::vector<T> src(v, v + n);
    for (size_t i = 0; i < n; ++i) {
        size_t j = (o & 0x80000000u) ? n - 1 - i : i;
        j = (j + (size_t)(o & 0x7fffffffu) % n) % n;
        v[j] = src[i];
    }
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Words per row: the fewest words of at most 32 bits such that every word
// holds a whole number of 4-site random-word blocks.
int words_per_row(int R) { return ea::words_per_row_c(R); }

// Any packing of a row of R sites into rw words of whole 4-site blocks, at
// most 32 sites per word.
bool rw_valid(int R, int rw) { return rw >= 1 && R % 4 == 0 && (R / 4) % rw == 0 && R / rw <= 32; }

// Packing of the plain form for side L when the caller leaves it open: the
// autotuned one (ea_tune_plain, or a line of the EA_TUNE_CACHE file), else
// the coarsest packing refined until one half-step launch has at least
// kPlainMinThreads threads (one wave per SIMD of every CU): below that a
// launch lasts as long as one thread's chain of dependent instructions.
constexpr long kPlainMinThreads = 65536;
constexpr int kMaxShellL = 256;      // largest side with full-vector C4 (its cost grows as L^6 / 64)
constexpr int kMaxShellLNoAlloc = 128;  // largest side of the allocation-free variant (its static scratch)
std::mutex g_plain_mu;
std::map<int, int> g_plain_tuned;  // L -> words per row
bool g_plain_file_read = false;

std::string device_arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// Lines "<arch> plain <L> <rw> <ms>" of the tuning cache (caller holds g_plain_mu).
void read_plain_tune_file()
{
    if (g_plain_file_read) return;
    g_plain_file_read = true;
    const char *path = std::getenv("EA_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    const std::string arch = device_arch_name();
    char line[256], a[64], tag[16];
    int L, rw;
    while (std::fgets(line, sizeof line, f))
        if (std::sscanf(line, "%63s %15s %d %d", a, tag, &L, &rw) == 4 && arch == a && std::string(tag) == "plain" &&
            L >= 8 && L <= kMaxL && L % 8 == 0 && rw_valid(L / 2, rw))
            g_plain_tuned[L] = rw;
    std::fclose(f);
}

// Whether the persistent slab path can run a lattice of side L in this
// packing: one z-plane of one colour (L rw words) must fit one workgroup's
// threads.
bool slab_capable(int L, int rw) { return L * rw <= ea::kSlabThreads; }

// Modelled time per sweep (us) of a plan whose workgroups own at most s
// planes each, used to pick one, with constants measured on MI355X.  A
// workgroup updates 1024 / (L rw) planes at once; in each such round its
// waves share the four SIMDs, and a SIMD runs the dependent chains of its
// waves' words about one after the other, one chain being ~(13.2 W + 40)
// instructions at ~4 cycles each.  With g = 1 a half-step costs ~0.9 us of
// exchange and barrier beyond its rounds; a cycle of g >= 2 half-steps costs
// ~3 us beyond its rounds (the ghost planes are read only after the
// neighbours' whole cycle, with a barrier on either side).  Measured per
// sweep against the model: L = 64 one plane of 4 words of 8 sites 2.36 us
// (2.29), L = 96 one plane of 2 words 2.97 (2.99) and of 3 words 3.34
// (3.48), L = 128 one plane 3.41 (3.34), five L = 128 runs on shares of 5
// planes 9.96 (9.50).
double slab_model_us(int L, int rw, int s, int g)
{
    const int W = L / 2 / rw, PL = L * rw;
    const double chain = (13.2 * W + 40.0) * 4.0 / 2400.0;  // one word's chain on a SIMD, us
    const int zstep = std::max(1, ea::kSlabThreads / PL);
    auto planes_us = [&](int n) {
        double t = 0.0;
        for (int left = n; left > 0; left -= zstep) {
            const int waves = (std::min(left, zstep) * PL + 63) / 64;
            t += (double)((waves + 3) / 4) * chain;
        }
        return t;
    };
    if (g == 1) return 2.0 * (0.9 + planes_us(s));
    double cycle = 3.0;
    for (int k = 1; k <= g; ++k) cycle += planes_us(s + 2 * g - 2 * k);
    return 2.0 * cycle / g;
}

double slab_best_model_us(int L, int rw)
{
    if (!slab_capable(L, rw)) return -1.0;
    double best = -1.0;
    for (int K = 1; K <= L && 2 * K <= 256; ++K)
        for (int g = 1; g <= 4; ++g) {
            const int emax = (L + K - 1) / K + 2 * g;
            if (4 * (8 * (size_t)emax * (size_t)(L * rw) + 16) > 160 * 1024 - 4 * (size_t)ea::kSelectTableWords)
                continue;
            const double c = slab_model_us(L, rw, (L + K - 1) / K, g);
            if (best < 0.0 || c < best) best = c;
        }
    return best;
}

// Default packing: for lattices that run as slabs the packing whose best
// slab plan the model rates fastest, a finer one only if it is rated 5%
// faster than a coarser one (grouped runs, whose slabs are thicker, do best
// with the coarsest); otherwise the coarsest packing refined until one
// half-step launch has at least kPlainMinThreads threads.
int plain_default_rw(int L)
{
    const int R = L / 2;
    int best_rw = 0;
    double best = 0.0;
    for (int d = 1; d <= R / 4; ++d) {
        if (!rw_valid(R, d)) continue;
        const double c = slab_best_model_us(L, d);
        if (c >= 0.0 && (best_rw == 0 || c < 0.95 * best)) {
            best = c;
            best_rw = d;
        }
    }
    if (best_rw) return best_rw;
    int rw = words_per_row(R);
    for (int d = rw + 1; d <= R / 4 && 2 * (long)L * L * rw < kPlainMinThreads; ++d)
        if (rw_valid(R, d)) rw = d;
    return rw;
}

int plain_rw(int L)
{
    std::lock_guard<std::mutex> lk(g_plain_mu);
    read_plain_tune_file();
    auto it = g_plain_tuned.find(L);
    return it != g_plain_tuned.end() ? it->second : plain_default_rw(L);
}

struct Layout {
    int L, R, RW, W, rows, plane;
    size_t spin_words, bond_words, snap_words, meas_count, xbuf_entries;
    size_t off_spins, off_bonds, off_snaps, off_meas, off_ctl, off_xbuf, total;
};

// Control words (in the 256-byte control area).
constexpr size_t kCtlTime = 0;   // uint32 sweep counter base of the captured graph
constexpr size_t kCtlErr = 64;   // uint32 error word of the slab launches

Layout make_layout(int L, int n_slots, int rw)
{
    Layout y{};
    y.L = L;
    y.R = L / 2;
    y.RW = rw;
    y.W = y.R / y.RW;
    y.rows = L * L;
    y.plane = y.rows * y.RW;
    y.spin_words = 4 * (size_t)y.plane;
    y.bond_words = 6 * (size_t)y.plane;
    y.snap_words = (size_t)n_slots * y.spin_words;
    y.meas_count = ea::M_AUTO + 2 * (size_t)kMaxSlots + 3 * (size_t)(y.R + 1);
    y.off_spins = 0;
    y.off_bonds = align256(y.off_spins + 4 * y.spin_words);
    y.off_snaps = align256(y.off_bonds + 4 * y.bond_words);
    y.off_meas = align256(y.off_snaps + 4 * y.snap_words);
    y.off_ctl = align256(y.off_meas + 8 * y.meas_count);
    // slab exchange entries: [replica][slot][colour][plane] 64-bit words
    y.xbuf_entries = slab_capable(L, rw) ? (size_t)ea::kSlabSlots * 4 * (size_t)y.plane : 0;
    y.off_xbuf = align256(y.off_ctl + 256);
    y.total = align256(y.off_xbuf + 8 * y.xbuf_entries);
    return y;
}

bool valid_L(int L) { return L >= 8 && L <= kMaxL && L % 8 == 0; }

}  // namespace

struct ea_sim {
    Layout lay;
    double p = 0, T = 0;
    uint64_t seed = 0;
    uint32_t sample = 0;
    int n_slots = 0;
    uint32_t thr[3] = {0, 0, 0};
    uint64_t pcut = 0;
    uint64_t t = 0;
    std::vector<uint64_t> snap_t;
    std::vector<char> snap_taken;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *buf = nullptr;
    bool own_buf = false;
    ea::Lattice lat{};
    uint32_t *snaps = nullptr;
    unsigned long long *meas = nullptr;
    uint32_t *t_dev = nullptr;  // device copy of the sweep counter base
    std::vector<unsigned long long> host_meas;
    // captured graph of kGraphSweeps sweeps (built on first use)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    uint32_t graph_order = 0;  // debug order the graph was captured with
    // scratch of ea_c4_shells (allocated on first use): dense rows and
    // shells, and the FFT route's complex array
    unsigned long long *c4_scratch = nullptr;
    void *fft_work = nullptr;
    // event ordering this run's stream with a group sweep (created on first use)
    hipEvent_t group_event = nullptr;
    // persistent slab path: plan (slabs per replica: 0 automatic, -1 off;
    // ghost planes: 0 automatic), exchange entries and their epoch serial
    int32_t slab_K = 0, slab_g = 0;
    unsigned long long *xbuf = nullptr;
    uint64_t xserial = 0;
    bool xbuf_clean = false;
    bool slab_used = false;
    uint32_t *err_dev = nullptr;
    int device = 0;  // the device current at ea_create

    ea::Geom geom() const
    {
        ea::Geom g;
        g.L = lay.L;
        g.R = lay.R;
        g.RW = lay.RW;
        g.rows = lay.rows;
        g.plane = lay.plane;
        g.order = debug_grid_order();
        return g;
    }
};

namespace {

uint32_t key_lo(const ea_sim *s) { return (uint32_t)(s->seed & 0xffffffffu); }
uint32_t key_hi(const ea_sim *s) { return (uint32_t)(s->seed >> 32); }

unsigned blocks_for(size_t n, unsigned bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// Dispatch a runtime word width to the kernel template instantiated for it.
#define EA_DISPATCH_W(W, ...)                                             \
    switch (W) {                                                          \
    case 4: { constexpr int WW = 4; __VA_ARGS__; } break;                 \
    case 8: { constexpr int WW = 8; __VA_ARGS__; } break;                 \
    case 12: { constexpr int WW = 12; __VA_ARGS__; } break;               \
    case 16: { constexpr int WW = 16; __VA_ARGS__; } break;               \
    case 20: { constexpr int WW = 20; __VA_ARGS__; } break;               \
    case 24: { constexpr int WW = 24; __VA_ARGS__; } break;               \
    case 28: { constexpr int WW = 28; __VA_ARGS__; } break;               \
    case 32: { constexpr int WW = 32; __VA_ARGS__; } break;               \
    default: return fail(EA_ERR_STATE, "unsupported word width %d", W);  \
    }

ea_status launch_init_lattice(const ea::Lattice &lat, const ea::Geom &g, int W, uint64_t seed, uint32_t sample,
                              uint64_t pcut, hipStream_t stream)
{
    dim3 grid(blocks_for(g.plane), 5, 2);
    EA_DISPATCH_W(W, hipLaunchKernelGGL((ea::init_kernel<WW>), grid, dim3(256), 0, stream, lat, g,
                                        (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), sample, pcut));
    EA_HIP(hipGetLastError());
    return EA_OK;
}

ea_status launch_init(ea_sim *s)
{
    return launch_init_lattice(s->lat, s->geom(), s->lay.W, s->seed, s->sample, s->pcut, s->stream);
}

// Half-step launches with at least this many threads (four waves per SIMD
// on 256 CUs) screen the rare uphill moves (ea::accept_screened); smaller
// ones are bound by one wave's latency and keep the plain select.
constexpr long kScreenThreads = 262144;

int screen_for(long threads) { return threads >= kScreenThreads ? 1 : 0; }

ea_status launch_half_step(ea_sim *s, int half, uint32_t t_off)
{
    ea::Geom g = s->geom();
    dim3 grid(blocks_for(g.plane), 2, 1);
    if (screen_for(2L * g.plane)) {
        EA_DISPATCH_W(s->lay.W,
                      hipLaunchKernelGGL((ea::half_step_kernel<WW, true>), grid, dim3(256), 0, s->stream, s->lat,
                                          g, half, s->t_dev, t_off, key_lo(s), key_hi(s), s->sample, s->thr[0],
                                          s->thr[1], s->thr[2]));
    } else {
        EA_DISPATCH_W(s->lay.W,
                      hipLaunchKernelGGL((ea::half_step_kernel<WW, false>), grid, dim3(256), 0, s->stream, s->lat,
                                          g, half, s->t_dev, t_off, key_lo(s), key_hi(s), s->sample, s->thr[0],
                                          s->thr[1], s->thr[2]));
    }
    return EA_OK;
}

// Sweeps per captured graph: long enough to amortise the replay, short
// enough that the remainder loop stays small.
constexpr uint32_t kGraphSweeps = 64;

// Enqueue sweeps t_dev + 0 .. t_dev + n-1 as plain launches.
ea_status launch_sweeps(ea_sim *s, uint32_t n)
{
    for (uint32_t i = 0; i < n; ++i) {
        ea_status st = launch_half_step(s, 0, i);
        if (st != EA_OK) return st;
        st = launch_half_step(s, 1, i);
        if (st != EA_OK) return st;
    }
    return EA_OK;
}

// Capture kGraphSweeps sweeps followed by the counter advance.
ea_status build_graph(ea_sim *s)
{
    s->graph_order = debug_grid_order();
    EA_HIP(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    ea_status st = launch_sweeps(s, kGraphSweeps);
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

// ---------------------------------------------------------------------------
// Persistent slab path (ea_slab_kernels.h).  A plan cuts each replica into K
// z-slabs, one workgroup each, with g ghost planes per side (g half-steps per
// exchange).  Every workgroup of a launch must be resident at once, so the
// grid never exceeds what the device holds; with work of other streams on
// the device a launch may wait for compute units, and a launch that cannot
// become whole within seconds ends with the error word set.

constexpr uint32_t kSlabMaxSweeps = 16384;  // sweeps per launch (a launch stays well under a second)
constexpr int kSlabMaxGhost = 8;

// A launch plan: B workgroups share the replicas' planes laid end to end
// (ea_slab_kernels.h), g ghost planes per side; K = B / (2 runs) when every
// workgroup holds one slab of one replica (explicit plans always do).
struct SlabPlan {
    int K = 0, B = 0, g = 0, emax = 0;
    size_t lds = 0;  // dynamic LDS bytes without a second select table
};

// Largest extended region (LDS planes) of any workgroup of a plan, computed
// as the kernel splits the shares.
int slab_emax(int L, int n_runs, int B, int g)
{
    const long P = 2L * n_runs * L;
    int emax = 0;
    for (int b = 0; b < B; ++b) {
        const int start = (int)((long)b * P / B), end = (int)((long)(b + 1) * P / B);
        const int cut = (start / L + 1) * L;
        const int e = end <= cut ? end - start + 2 * g : (cut - start + 2 * g) + (end - cut + 2 * g);
        emax = std::max(emax, e);
    }
    return emax;
}

size_t slab_lds_bytes(int L, int rw, int emax) { return 4 * (8 * (size_t)emax * (size_t)(L * rw) + 16); }

std::mutex g_slab_mu;
int g_slab_cus = 0, g_slab_lds_limit = 0;
bool g_slab_attr[33] = {};

template <bool SCREEN, bool SPAN>
const void *slab_kernel_fn(int W)
{
    switch (W) {
    case 4: return (const void *)ea::slab_sweep_kernel<4, SCREEN, SPAN>;
    case 8: return (const void *)ea::slab_sweep_kernel<8, SCREEN, SPAN>;
    case 12: return (const void *)ea::slab_sweep_kernel<12, SCREEN, SPAN>;
    case 16: return (const void *)ea::slab_sweep_kernel<16, SCREEN, SPAN>;
    case 20: return (const void *)ea::slab_sweep_kernel<20, SCREEN, SPAN>;
    case 24: return (const void *)ea::slab_sweep_kernel<24, SCREEN, SPAN>;
    case 28: return (const void *)ea::slab_sweep_kernel<28, SCREEN, SPAN>;
    default: return (const void *)ea::slab_sweep_kernel<32, SCREEN, SPAN>;
    }
}

// Compute units and the dynamic LDS a slab workgroup may use beside the
// static select tables (queried once), and the kernel attribute that lets
// the instantiations for width W use all of it.
ea_status slab_device(int W, int *n_cu, int *lds_limit)
{
    std::lock_guard<std::mutex> lk(g_slab_mu);
    if (!g_slab_cus) {
        int dev = 0, per_block = 0;
        EA_HIP(hipGetDevice(&dev));
        EA_HIP(hipDeviceGetAttribute(&g_slab_cus, hipDeviceAttributeMultiprocessorCount, dev));
        EA_HIP(hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        g_slab_lds_limit = per_block - 4 * ea::kSelectTableWords;
    }
    if (W < 4 || W > 32 || W % 4) return fail(EA_ERR_STATE, "unsupported word width %d", W);
    if (!g_slab_attr[W]) {
        const void *fns[4] = {slab_kernel_fn<false, false>(W), slab_kernel_fn<true, false>(W),
                              slab_kernel_fn<false, true>(W), slab_kernel_fn<true, true>(W)};
        for (const void *fn : fns)
            EA_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, g_slab_lds_limit));
        g_slab_attr[W] = true;
    }
    *n_cu = g_slab_cus;
    *lds_limit = g_slab_lds_limit;
    return EA_OK;
}

// A plan of B workgroups (g > 1: whole slabs only, B = 2 runs K) if it fits
// the device: at most one 1024-thread workgroup per compute unit, shares
// within one replica's length, the extended regions within the LDS.
bool slab_plan_fits(int L, int rw, int n_runs, int B, int g, int n_cu, int lds_limit, SlabPlan *out)
{
    const long P = 2L * n_runs * L;
    if (B < 2 * n_runs || B > P || B > n_cu || g < 1 || g > kSlabMaxGhost || g > L) return false;
    const bool whole = B % (2 * n_runs) == 0;
    if (g > 1 && !whole) return false;
    const int emax = slab_emax(L, n_runs, B, g);
    const size_t lds = slab_lds_bytes(L, rw, emax);
    // shares that span two runs may need a second select table
    const size_t extra = (!whole && n_runs > 1) ? 4 * (size_t)ea::kSelectTableWords : 0;
    if (lds + extra > (size_t)lds_limit) return false;
    out->K = whole ? B / (2 * n_runs) : 0;
    out->B = B;
    out->g = g;
    out->emax = emax;
    out->lds = lds;
    return true;
}

// The plan for n_runs runs of side L in packing rw: the requested slabs per
// replica (K > 0; g = 0 picks the best ghost depth for it), else the
// modelled best, where shares of g = 1 plans may span two replicas (an even
// number of workgroups).
ea_status slab_choose(int L, int rw, int n_runs, int K_req, int g_req, SlabPlan *plan)
{
    if (!slab_capable(L, rw)) return fail(EA_ERR_ARG, "L=%d with %d words per row has no slab plan", L, rw);
    int n_cu = 0, lds_limit = 0;
    ea_status st = slab_device(L / 2 / rw, &n_cu, &lds_limit);
    if (st != EA_OK) return st;
    const long P = 2L * n_runs * L;
    double best = 0.0;
    bool found = false;
    auto consider = [&](int B, int g) {
        SlabPlan p;
        if (!slab_plan_fits(L, rw, n_runs, B, g, n_cu, lds_limit, &p)) return;
        const double c = slab_model_us(L, rw, (int)((P + B - 1) / B), g);
        if (!found || c < best) {
            best = c;
            *plan = p;
            found = true;
        }
    };
    const int g_lo = g_req > 0 ? g_req : 1, g_hi = g_req > 0 ? g_req : 4;
    if (K_req > 0) {
        if (K_req <= L)
            for (int g = g_lo; g <= g_hi; ++g) consider(2 * n_runs * K_req, g);
    } else {
        for (int g = g_lo; g <= g_hi; ++g) {
            if (g == 1)
                for (int B = 2 * n_runs; B <= n_cu && B <= P; B += 2) consider(B, 1);
            else
                for (int K = 1; K <= L; ++K) consider(2 * n_runs * K, g);
        }
    }
    if (!found)
        return fail(EA_ERR_ARG, "no slab plan (K=%d, g=%d) fits %d run(s) of L=%d on %d compute units", K_req,
                    g_req, n_runs, L, n_cu);
    return EA_OK;
}

// The plan a run uses alone (K = -1: the slab path is off for it).
ea_status slab_plan_of(const ea_sim *s, int n_runs, SlabPlan *plan)
{
    if (s->slab_K < 0 || !slab_capable(s->lay.L, s->lay.RW)) {
        plan->K = -1;
        return EA_OK;
    }
    return slab_choose(s->lay.L, s->lay.RW, n_runs, s->slab_K, s->slab_g, plan);
}

// Advance runs[0..n) (same L and packing, at most kGroupMax) by n sweeps with
// slab launches on the first run's stream.
ea_status launch_slab(ea_sim *const *runs, int n, uint64_t sweeps, const SlabPlan &plan)
{
    ea_sim *lead = runs[0];
    const Layout &y = lead->lay;
    for (int i = 0; i < n; ++i) {
        ea_sim *m = runs[i];
        if (!m->xbuf_clean) {  // entries of no earlier epoch
            hipLaunchKernelGGL(ea::zero_u64_kernel, dim3(blocks_for(y.xbuf_entries)), dim3(256), 0, lead->stream,
                               m->xbuf, y.xbuf_entries);
            m->xbuf_clean = true;
            m->xserial = 0;
        }
        m->slab_used = true;
    }
    // a second select table when some workgroup's two pieces belong to runs
    // of different temperature
    int tables = 1;
    bool span = false;  // some share holds two pieces: the two-piece instantiation
    for (int b = 0; b < plan.B; ++b) {
        const long P = 2L * n * y.L;
        const int start = (int)((long)b * P / plan.B), end = (int)((long)(b + 1) * P / plan.B);
        const int q0 = start / y.L;
        if (end > (q0 + 1) * y.L) {
            span = true;
            const ea_sim *u = runs[q0 / 2], *v = runs[(q0 + 1) / 2];
            if (u->thr[0] != v->thr[0] || u->thr[1] != v->thr[1] || u->thr[2] != v->thr[2]) tables = 2;
        }
    }
    const size_t lds = plan.lds + (tables == 2 ? 4 * (size_t)ea::kSelectTableWords : 0);
    uint64_t done = 0;
    while (done < sweeps) {
        const uint32_t chunk = (uint32_t)std::min<uint64_t>(kSlabMaxSweeps, sweeps - done);
        ea::SlabLaunch a{};
        a.L = y.L;
        a.RW = y.RW;
        a.g = plan.g;
        a.B = plan.B;
        a.P = 2 * n * y.L;
        a.emax = plan.emax;
        a.tables = tables;
        a.n_half = 2 * chunk;
        a.err = lead->err_dev;
        a.order = debug_grid_order();
        a.poison = debug_poison_word();
        const uint64_t n_cycles = (a.n_half + (uint64_t)plan.g - 1) / (uint64_t)plan.g;
        for (int i = 0; i < n; ++i) {
            ea_sim *m = runs[i];
            if ((m->xserial & 0xffffffffull) + n_cycles + 2 >= (1ull << 32)) {
                // the 32-bit epochs would wrap: start over from cleared entries
                hipLaunchKernelGGL(ea::zero_u64_kernel, dim3(blocks_for(y.xbuf_entries)), dim3(256), 0,
                                   lead->stream, m->xbuf, y.xbuf_entries);
                m->xserial = 0;
            }
            ea::SlabRunDev &d = a.runs[i];
            d.spins = m->lat.spins;
            d.bonds = m->lat.bonds;
            d.xbuf = m->xbuf;
            d.k0 = key_lo(m);
            d.k1 = key_hi(m);
            d.sample = m->sample;
            d.thr1 = m->thr[0];
            d.thr2 = m->thr[1];
            d.thr3 = m->thr[2];
            d.t0 = (uint32_t)(m->t + done);
            d.serial = (uint32_t)m->xserial;
            m->xserial += n_cycles + 1;
        }
        const dim3 grid((unsigned)plan.B);
        // the screen pays where every workgroup gives each SIMD four waves of work
        const bool screen = (long)(a.P / plan.B) * y.L * y.RW >= ea::kSlabThreads;
        if (screen && span) {
            EA_DISPATCH_W(y.W, hipLaunchKernelGGL((ea::slab_sweep_kernel<WW, true, true>), grid,
                                                  dim3(ea::kSlabThreads), lds, lead->stream, a));
        } else if (screen) {
            EA_DISPATCH_W(y.W, hipLaunchKernelGGL((ea::slab_sweep_kernel<WW, true, false>), grid,
                                                  dim3(ea::kSlabThreads), lds, lead->stream, a));
        } else if (span) {
            EA_DISPATCH_W(y.W, hipLaunchKernelGGL((ea::slab_sweep_kernel<WW, false, true>), grid,
                                                  dim3(ea::kSlabThreads), lds, lead->stream, a));
        } else {
            EA_DISPATCH_W(y.W, hipLaunchKernelGGL((ea::slab_sweep_kernel<WW, false, false>), grid,
                                                  dim3(ea::kSlabThreads), lds, lead->stream, a));
        }
        EA_HIP(hipGetLastError());
        done += chunk;
    }
    // the launch-wide error word is the lead's; the others copy it
    for (int i = 1; i < n; ++i)
        hipLaunchKernelGGL(ea::or_word_kernel, dim3(1), dim3(64), 0, lead->stream, runs[i]->err_dev, lead->err_dev);
    EA_HIP(hipGetLastError());
    return EA_OK;
}

// After a synchronisation: EA_ERR_DEVICE if a slab launch of the run gave up
// waiting for a neighbouring slab (the run's state is then undefined until
// ea_reset).
ea_status slab_check(ea_sim *s)
{
    if (!s->slab_used) return EA_OK;
    uint32_t e = 0;
    EA_HIP(hipMemcpy(&e, s->err_dev, 4, hipMemcpyDeviceToHost));
    if (e)
        return fail(EA_ERR_DEVICE, "a slab launch gave up waiting for a neighbouring slab (its workgroups were not "
                                   "all resident within seconds); the run's state is undefined until ea_reset");
    return EA_OK;
}

// Shell sums of dense overlap rows (ea_shells.h) for any L up to 256.
ea_status launch_shell_rows(const unsigned long long *qd, int L, int n_shells, unsigned long long *shells,
                            hipStream_t stream)
{
    const dim3 grid((unsigned)((L + ea::kShellChunk - 1) / ea::kShellChunk), (unsigned)(L * L));
    switch ((L + 63) / 64) {
    case 1: hipLaunchKernelGGL((ea::c4_shell_rows_kernel<1>), grid, dim3(256), 0, stream, qd, L, n_shells, shells); break;
    case 2: hipLaunchKernelGGL((ea::c4_shell_rows_kernel<2>), grid, dim3(256), 0, stream, qd, L, n_shells, shells); break;
    case 3: hipLaunchKernelGGL((ea::c4_shell_rows_kernel<3>), grid, dim3(256), 0, stream, qd, L, n_shells, shells); break;
    case 4: hipLaunchKernelGGL((ea::c4_shell_rows_kernel<4>), grid, dim3(256), 0, stream, qd, L, n_shells, shells); break;
    default: return fail(EA_ERR_ARG, "full-vector C4 needs L <= 256 (L=%d)", L);
    }
    EA_HIP(hipGetLastError());
    return EA_OK;
}

// Route of the full-vector C4 shells (ea_set_shell_route).
std::atomic<int32_t> g_shell_route{EA_SHELLS_AUTO};
// automatic route: FFT for L = 2^k or 3 2^k from this side on (at L = 32 the
// direct kernel is faster: 0.07 against 0.10 ms per call)
constexpr int kFftAutoMinL = 64;

bool shells_by_fft(int L)
{
    const int32_t r = g_shell_route.load();
    if (!ea::fft_side(L) || r == EA_SHELLS_DIRECT) return false;
    return r == EA_SHELLS_FFT || L >= kFftAutoMinL;
}

// Device scratch of a handle's full-vector C4 calls (ea_batch_c4_shells,
// ea_msc_c4_shells): allocated on the first call, grown when a call needs
// more, freed with the handle.  The calls synchronise before they return, so
// the next call may reuse it.
struct ShellScratch {
    void *p = nullptr;
    size_t bytes = 0;
    ShellScratch() = default;
    ShellScratch(const ShellScratch &) = delete;
    ShellScratch &operator=(const ShellScratch &) = delete;
    ~ShellScratch()
    {
        if (p) (void)hipFree(p);
    }
    ea_status reserve(size_t n)
    {
        if (n <= bytes) return EA_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        const hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(EA_ERR_NOMEM, "hipMalloc(C4 shell scratch, %zu bytes): %s", n, hipGetErrorString(e));
        }
        bytes = n;
        return EA_OK;
    }
};

// Device bytes of the FFT route: the complex array, then the error word.
size_t fft_work_bytes(int L) { return 16 * (size_t)L * L * L + 256; }

template <int L>
void launch_fft_passes(const ea::FftArgs &a, hipStream_t stream)
{
    constexpr int H = L / 2, B = ea::FftShape<L>::B;
    const dim3 grid((unsigned)(L * L / B)), block(ea::kFftThreads);
    const dim3 half((unsigned)((H + 1) * (L / B)));  // tiles of the planes z <= L/2
    const dim3 bins((unsigned)((H + 1) * ((H + ea::kFftBinY) / ea::kFftBinY)));
    hipLaunchKernelGGL((ea::fft_pass_kernel<L, ea::kFftFwdBitsX>), grid, block, 0, stream, a);
    hipLaunchKernelGGL((ea::fft_pass_kernel<L, ea::kFftFwdY>), grid, block, 0, stream, a);
    hipLaunchKernelGGL((ea::fft_pass_kernel<L, ea::kFftSquareZ>), grid, block, 0, stream, a);
    hipLaunchKernelGGL((ea::fft_pass_kernel<L, ea::kFftInvY>), half, block, 0, stream, a);
    hipLaunchKernelGGL((ea::fft_bin_kernel<L>), bins, block, 0, stream, a);
    hipLaunchKernelGGL((ea::fft_shell_sum_kernel<L>), dim3(blocks_for((size_t)(H + 1) * (H + 1) * (H + 1))),
                       dim3(256), 0, stream, a);
}

// Shell sums of dense overlap rows (dw words per row) through the FFT route
// (ea_fft.h), added to `shells`; `work` holds fft_work_bytes(L) bytes.
ea_status launch_fft_shells(const unsigned long long *qd, int dw, int L, int n_shells, unsigned long long *shells,
                            void *work, hipStream_t stream)
{
    ea::FftArgs a{};
    a.z = (double2 *)work;
    a.qd = qd;
    a.dw = dw;
    a.n_shells = n_shells;
    a.shells = shells;
    unsigned long long *err = (unsigned long long *)((char *)work + 16 * (size_t)L * L * L);
    a.err = (unsigned int *)err;
    hipLaunchKernelGGL(ea::zero_u64_kernel, dim3(1), dim3(256), 0, stream, err, (size_t)1);
    switch (L) {
    case 8: launch_fft_passes<8>(a, stream); break;
    case 16: launch_fft_passes<16>(a, stream); break;
    case 32: launch_fft_passes<32>(a, stream); break;
    case 64: launch_fft_passes<64>(a, stream); break;
    case 128: launch_fft_passes<128>(a, stream); break;
    case 256: launch_fft_passes<256>(a, stream); break;
    case 24: launch_fft_passes<24>(a, stream); break;
    case 48: launch_fft_passes<48>(a, stream); break;
    case 96: launch_fft_passes<96>(a, stream); break;
    case 192: launch_fft_passes<192>(a, stream); break;
    default: return fail(EA_ERR_ARG, "the FFT route of full-vector C4 needs L = 2^k or 3 2^k in 8..256 (L=%d)", L);
    }
    EA_HIP(hipGetLastError());
    return EA_OK;
}

// After the stream has passed launch_fft_shells: EA_ERR_DEVICE if a sum was
// not within 1/4 of an integer (it never is within the fp64 error bound).
ea_status fft_shells_check(const void *work, int L, hipStream_t stream)
{
    uint32_t e = 0;
    EA_HIP(hipMemcpyAsync(&e, (const char *)work + 16 * (size_t)L * L * L, 4, hipMemcpyDeviceToHost, stream));
    EA_HIP(hipStreamSynchronize(stream));
    if (e) return fail(EA_ERR_DEVICE, "full-vector C4 (FFT route, L=%d): a correlation sum was not an integer", L);
    return EA_OK;
}

void host_thresholds(double T, uint32_t out[3])
{
    for (int k = 1; k <= 3; ++k) {
        if (!(T > 0.0)) {
            out[k - 1] = 0;
            continue;
        }
        const double v = std::floor(std::exp(-4.0 * k / T) * 4294967296.0);
        out[k - 1] = v >= 4294967295.0 ? 0xffffffffu : (uint32_t)v;
    }
}

// Host-side conversion between canonical int8 +-1 arrays and packed planes.
struct SiteAddr {
    int c;
    size_t word;
    int bit;
};

SiteAddr address_of(const Layout &y, int64_t s)
{
    const int L = y.L;
    const int x = (int)(s % L), yy = (int)((s / L) % L), z = (int)(s / ((int64_t)L * L));
    SiteAddr a;
    a.c = (x + yy + z) & 1;
    const int xh = x >> 1;
    const int row = yy + L * z;
    a.word = (size_t)row * y.RW + (size_t)(xh / y.W);
    a.bit = xh % y.W;
    return a;
}

}  // namespace

extern "C" {

const char *ea_last_error(void) { return g_last_error.c_str(); }

const char *ea_version(void) { return "ea-mi355x 0.1 (gfx950)"; }

ea_status ea_footprint(int32_t L, int32_t n_tw, size_t *bytes)
{
    if (!bytes) return fail(EA_ERR_ARG, "bytes is NULL");
    if (!valid_L(L)) return fail(EA_ERR_ARG, "L=%d must be a multiple of 8 in [8, %d]", L, kMaxL);
    if (n_tw < 0 || n_tw > kMaxSlots) return fail(EA_ERR_ARG, "n_tw=%d outside [0, %d]", n_tw, kMaxSlots);
    *bytes = make_layout(L, n_tw, plain_rw(L)).total;
    return EA_OK;
}

ea_status ea_footprint_ex(const ea_config *cfg, size_t *bytes)
{
    if (!cfg || !bytes) return fail(EA_ERR_ARG, "NULL argument");
    if (!valid_L(cfg->L)) return fail(EA_ERR_ARG, "L=%d must be a multiple of 8 in [8, %d]", cfg->L, kMaxL);
    if (cfg->n_tw_slots < 0 || cfg->n_tw_slots > kMaxSlots)
        return fail(EA_ERR_ARG, "n_tw_slots=%d outside [0, %d]", cfg->n_tw_slots, kMaxSlots);
    const int rw = cfg->words_per_row ? cfg->words_per_row : plain_rw(cfg->L);
    if (!rw_valid(cfg->L / 2, rw)) return fail(EA_ERR_ARG, "invalid words_per_row=%d", rw);
    *bytes = make_layout(cfg->L, cfg->n_tw_slots, rw).total;
    return EA_OK;
}

ea_status ea_words_per_row(const ea_sim *s, int32_t *rw)
{
    if (!s || !rw) return fail(EA_ERR_ARG, "NULL argument");
    *rw = s->lay.RW;
    return EA_OK;
}

ea_status ea_thresholds(double T, uint32_t out[3])
{
    if (!out) return fail(EA_ERR_ARG, "out is NULL");
    if (!(T >= 0.0) || !std::isfinite(T)) return fail(EA_ERR_ARG, "T=%g must be finite and >= 0", T);
    host_thresholds(T, out);
    return EA_OK;
}

ea_status ea_set_debug(uint32_t flags, uint32_t seed)
{
    const uint32_t known = EA_DEBUG_REVERSE | EA_DEBUG_ROTATE | EA_DEBUG_POISON;
    if (flags & ~known) return fail(EA_ERR_ARG, "unknown debug flags 0x%x", flags & ~known);
    g_debug_seed.store(seed);
    g_debug_flags.store(flags);
    return EA_OK;
}

ea_status ea_get_debug(uint32_t *flags, uint32_t *seed)
{
    if (!flags || !seed) return fail(EA_ERR_ARG, "NULL argument");
    *flags = g_debug_flags.load();
    *seed = g_debug_seed.load();
    return EA_OK;
}

ea_status ea_create(int32_t L, double p, double T, uint64_t seed, ea_sim **out)
{
    ea_config cfg{};
    cfg.L = L;
    cfg.p = p;
    cfg.T = T;
    cfg.seed = seed;
    return ea_create_ex(&cfg, out);
}

ea_status ea_create_ex(const ea_config *cfg, ea_sim **out)
{
    if (!cfg || !out) return fail(EA_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (!valid_L(cfg->L)) return fail(EA_ERR_ARG, "L=%d must be a multiple of 8 in [8, %d]", cfg->L, kMaxL);
    if (!(cfg->p >= 0.0 && cfg->p <= 1.0)) return fail(EA_ERR_ARG, "p=%g outside [0, 1]", cfg->p);
    if (!(cfg->T >= 0.0) || !std::isfinite(cfg->T))
        return fail(EA_ERR_ARG, "T=%g must be finite and >= 0", cfg->T);
    if (cfg->n_tw_slots < 0 || cfg->n_tw_slots > kMaxSlots)
        return fail(EA_ERR_ARG, "n_tw_slots=%d outside [0, %d]", cfg->n_tw_slots, kMaxSlots);

    const int rw = cfg->words_per_row ? cfg->words_per_row : plain_rw(cfg->L);
    if (!rw_valid(cfg->L / 2, rw))
        return fail(EA_ERR_ARG, "words_per_row=%d does not split a row of %d sites into whole 4-site blocks of "
                                "at most 32", rw, cfg->L / 2);
    Layout lay = make_layout(cfg->L, cfg->n_tw_slots, rw);
    if (cfg->dev_buf) {
        if (cfg->dev_buf_bytes < lay.total)
            return fail(EA_ERR_ARG, "dev_buf holds %zu bytes, %zu needed", cfg->dev_buf_bytes, lay.total);
        if (((uintptr_t)cfg->dev_buf & 255) != 0) return fail(EA_ERR_ARG, "dev_buf is not 256-byte aligned");
    }

    ea_sim *s = new (std::nothrow) ea_sim();
    if (!s) return fail(EA_ERR_NOMEM, "host allocation failed");
    s->lay = lay;
    s->p = cfg->p;
    s->T = cfg->T;
    s->seed = cfg->seed;
    s->sample = cfg->sample;
    s->n_slots = cfg->n_tw_slots;
    s->snap_t.assign((size_t)s->n_slots, 0);
    s->snap_taken.assign((size_t)s->n_slots, 0);
    s->host_meas.assign(lay.meas_count, 0);
    host_thresholds(cfg->T, s->thr);
    s->pcut = (uint64_t)std::floor(std::ldexp(cfg->p, 32));

    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return fail(EA_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
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
        e = hipMalloc((void **)&s->buf, lay.total);
        if (e != hipSuccess) {
            ea_destroy(s);
            return fail(EA_ERR_NOMEM, "hipMalloc(%zu): %s", lay.total, hipGetErrorString(e));
        }
        s->own_buf = true;
    }
    s->lat.spins = (uint32_t *)(s->buf + lay.off_spins);
    s->lat.bonds = (uint32_t *)(s->buf + lay.off_bonds);
    s->snaps = (uint32_t *)(s->buf + lay.off_snaps);
    s->meas = (unsigned long long *)(s->buf + lay.off_meas);
    s->t_dev = (uint32_t *)(s->buf + lay.off_ctl + kCtlTime);
    s->err_dev = (uint32_t *)(s->buf + lay.off_ctl + kCtlErr);
    s->xbuf = lay.xbuf_entries ? (unsigned long long *)(s->buf + lay.off_xbuf) : nullptr;
    hipLaunchKernelGGL(ea::zero_u32_kernel, dim3(1), dim3(64), 0, s->stream, s->err_dev, (size_t)1);

    ea_status st = launch_init(s);
    if (st != EA_OK) {
        ea_destroy(s);
        return st;
    }
    if (s->n_slots > 0) {
        hipLaunchKernelGGL(ea::zero_u64_kernel, dim3(blocks_for(lay.snap_words / 2)), dim3(256), 0, s->stream,
                           (unsigned long long *)s->snaps, lay.snap_words / 2);
    }
    *out = s;
    return EA_OK;
}

void ea_destroy(ea_sim *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->c4_scratch) (void)hipFree(s->c4_scratch);
    if (s->fft_work) (void)hipFree(s->fft_work);
    if (s->group_event) (void)hipEventDestroy(s->group_event);
    if (s->own_buf && s->buf) (void)hipFree(s->buf);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

ea_status ea_reset(ea_sim *s, uint64_t seed, uint32_t sample)
{
    if (!s) return fail(EA_ERR_ARG, "sim is NULL");
    s->seed = seed;
    s->sample = sample;
    s->t = 0;
    std::fill(s->snap_t.begin(), s->snap_t.end(), 0);
    std::fill(s->snap_taken.begin(), s->snap_taken.end(), 0);
    // the captured sweeps bake the key into their arguments
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->graph_exec = nullptr;
    s->graph = nullptr;
    hipLaunchKernelGGL(ea::zero_u32_kernel, dim3(1), dim3(64), 0, s->stream, s->err_dev, (size_t)1);
    return launch_init(s);
}

ea_status ea_sweep(ea_sim *s, uint64_t n)
{
    if (!s) return fail(EA_ERR_ARG, "sim is NULL");
    if (s->t + n >= (1ull << 32) || n >= (1ull << 32))
        return fail(EA_ERR_ARG, "t + n = %llu would reach 2^32", (unsigned long long)(s->t + n));
    if (n == 0) return EA_OK;
    SlabPlan plan;
    ea_status pst = slab_plan_of(s, 1, &plan);
    if (pst != EA_OK) return pst;
    if (plan.B > 0) {
        ea_sim *one[1] = {s};
        pst = launch_slab(one, 1, n, plan);
        if (pst != EA_OK) return pst;
        s->t += n;
        return EA_OK;
    }
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
            ea_status st = build_graph(s);
            if (st != EA_OK) return st;
        }
        for (; left >= kGraphSweeps; left -= kGraphSweeps) EA_HIP(hipGraphLaunch(s->graph_exec, s->stream));
        // the graph advanced the device counter by kGraphSweeps per replay
    }
    ea_status st = launch_sweeps(s, (uint32_t)left);
    if (st != EA_OK) return st;
    EA_HIP(hipGetLastError());
    s->t += n;
    return EA_OK;
}

namespace {

ea_status group_event(ea_sim *s)
{
    if (!s->group_event) EA_HIP(hipEventCreateWithFlags(&s->group_event, hipEventDisableTiming));
    return EA_OK;
}

}  // namespace

ea_status ea_sweep_group(ea_sim *const *sims, int32_t n_sims, uint64_t n)
{
    if (!sims || n_sims < 1) return fail(EA_ERR_ARG, "need at least one run");
    for (int32_t i = 0; i < n_sims; ++i) {
        if (!sims[i]) return fail(EA_ERR_ARG, "run %d is NULL", i);
        if (sims[i]->lay.L != sims[0]->lay.L || sims[i]->lay.RW != sims[0]->lay.RW)
            return fail(EA_ERR_ARG, "run %d: L=%d with %d words per row, run 0: L=%d with %d", i, sims[i]->lay.L,
                        sims[i]->lay.RW, sims[0]->lay.L, sims[0]->lay.RW);
        for (int32_t j = 0; j < i; ++j)
            if (sims[j] == sims[i]) return fail(EA_ERR_ARG, "run %d appears twice", i);
        if (sims[i]->t + n >= (1ull << 32) || n >= (1ull << 32))
            return fail(EA_ERR_ARG, "run %d: t + n would reach 2^32", i);
    }
    if (n == 0) return EA_OK;
    ea_sim *lead = sims[0];
    // the work runs on the first run's stream, after everything queued on the others
    for (int32_t i = 1; i < n_sims; ++i) {
        if (sims[i]->stream == lead->stream) continue;
        ea_status st = group_event(sims[i]);
        if (st != EA_OK) return st;
        EA_HIP(hipEventRecord(sims[i]->group_event, sims[i]->stream));
        EA_HIP(hipStreamWaitEvent(lead->stream, sims[i]->group_event, 0));
    }
    SlabPlan plan;
    {
        const int per = std::min<int32_t>(ea::kGroupMax, n_sims);
        ea_status pst = slab_plan_of(lead, per, &plan);
        if (pst != EA_OK) return pst;
    }
    if (plan.B > 0) {
        // one slab launch per chunk of at most kGroupMax runs
        for (int32_t c0 = 0; c0 < n_sims; c0 += ea::kGroupMax) {
            const int cnt = std::min<int32_t>(ea::kGroupMax, n_sims - c0);
            SlabPlan pc = plan;
            if (cnt != std::min<int32_t>(ea::kGroupMax, n_sims)) {
                ea_status pst = slab_plan_of(lead, cnt, &pc);
                if (pst != EA_OK) return pst;
            }
            ea_status st = launch_slab(sims + c0, cnt, n, pc);
            if (st != EA_OK) return st;
        }
    } else {
    ea::Geom g = lead->geom();
    for (int32_t i = 0; i < n_sims; ++i)
        hipLaunchKernelGGL(ea::set_u32_kernel, dim3(1), dim3(64), 0, lead->stream, sims[i]->t_dev,
                           (uint32_t)sims[i]->t);
    // member arguments, one block of at most kGroupMax runs per launch
    std::vector<ea::GroupArgs> chunks((size_t)((n_sims + ea::kGroupMax - 1) / ea::kGroupMax));
    for (int32_t i = 0; i < n_sims; ++i) {
        const ea_sim *m = sims[i];
        ea::GroupMember &gm = chunks[(size_t)(i / ea::kGroupMax)].m[i % ea::kGroupMax];
        gm.lat = m->lat;
        gm.t_base = m->t_dev;
        gm.k0 = key_lo(m);
        gm.k1 = key_hi(m);
        gm.sample = m->sample;
        gm.thr1 = m->thr[0];
        gm.thr2 = m->thr[1];
        gm.thr3 = m->thr[2];
    }
    // sweep by sweep, every chunk of runs for each half-step
    for (uint64_t k = 0; k < n; ++k)
        for (int half = 0; half < 2; ++half)
            for (size_t c = 0; c < chunks.size(); ++c) {
                const int32_t cnt = std::min<int32_t>(ea::kGroupMax, n_sims - (int32_t)c * ea::kGroupMax);
                const dim3 grid(blocks_for(g.plane), 2, (unsigned)cnt);
                if (screen_for(2L * g.plane * cnt)) {
                    EA_DISPATCH_W(lead->lay.W,
                                  hipLaunchKernelGGL((ea::group_half_step_kernel<WW, true>), grid, dim3(256), 0,
                                                     lead->stream, chunks[c], g, half, (uint32_t)k));
                } else {
                    EA_DISPATCH_W(lead->lay.W,
                                  hipLaunchKernelGGL((ea::group_half_step_kernel<WW, false>), grid, dim3(256), 0,
                                                     lead->stream, chunks[c], g, half, (uint32_t)k));
                }
            }
    }
    EA_HIP(hipGetLastError());
    ea_status st = group_event(lead);
    if (st != EA_OK) return st;
    EA_HIP(hipEventRecord(lead->group_event, lead->stream));
    for (int32_t i = 1; i < n_sims; ++i)
        if (sims[i]->stream != lead->stream) EA_HIP(hipStreamWaitEvent(sims[i]->stream, lead->group_event, 0));
    for (int32_t i = 0; i < n_sims; ++i) sims[i]->t += n;
    return EA_OK;
}

ea_status ea_snapshot(ea_sim *s, int32_t slot)
{
    if (!s) return fail(EA_ERR_ARG, "sim is NULL");
    if (slot < 0 || slot >= s->n_slots) return fail(EA_ERR_ARG, "slot %d outside [0, %d)", slot, s->n_slots);
    const size_t n = s->lay.spin_words;
    hipLaunchKernelGGL(ea::copy_words_kernel, dim3(blocks_for(n)), dim3(256), 0, s->stream,
                       s->snaps + (size_t)slot * n, s->lat.spins, n);
    EA_HIP(hipGetLastError());
    s->snap_t[(size_t)slot] = s->t;
    s->snap_taken[(size_t)slot] = 1;
    return EA_OK;
}

ea_status ea_measure(ea_sim *s, ea_obs *out)
{
    if (!s || !out) return fail(EA_ERR_ARG, "NULL argument");
    const Layout &y = s->lay;
    if (out->autocorr && out->n_tw != s->n_slots)
        return fail(EA_ERR_ARG, "n_tw=%d but the run has %d slots", out->n_tw, s->n_slots);
    if (out->c4 && out->rmax != y.R) return fail(EA_ERR_ARG, "rmax=%d but L/2=%d", out->rmax, y.R);
    ea::Geom g = s->geom();
    const size_t c4_base = ea::M_AUTO + 2 * (size_t)kMaxSlots;
    const size_t n_count = c4_base + 3 * (size_t)(y.R + 1);
    hipLaunchKernelGGL(ea::zero_u64_kernel, dim3(blocks_for(n_count)), dim3(256), 0, s->stream, s->meas, n_count);
    const int slots = out->autocorr ? s->n_slots : 0;
    EA_DISPATCH_W(y.W, hipLaunchKernelGGL((ea::measure_kernel<WW>), dim3(blocks_for(2 * (size_t)g.plane)),
                                           dim3(256), 0, s->stream, s->lat, g, s->snaps, slots, s->meas));
    if (out->c4) {
        dim3 grid(blocks_for(2 * (size_t)g.rows), 3 * (unsigned)ea::c4_chunks(y.R), 1);
        EA_DISPATCH_W(y.W, hipLaunchKernelGGL((ea::c4_kernel<WW>), grid, dim3(256), 0, s->stream,
                                               s->lat, g, s->meas + c4_base));
    }
    EA_HIP(hipGetLastError());
    EA_HIP(hipMemcpyAsync(s->host_meas.data(), s->meas, n_count * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));
    ea_status est = slab_check(s);
    if (est != EA_OK) return est;

    const int64_t N = (int64_t)y.L * y.L * y.L;
    const unsigned long long *m = s->host_meas.data();
    out->t = s->t;
    for (int r = 0; r < 2; ++r) {
        out->unsat[r] = (int64_t)m[ea::M_UNSAT + r];
        out->mag[r] = N - 2 * (int64_t)m[ea::M_DOWN + r];
    }
    out->overlap = N - 2 * (int64_t)m[ea::M_QDIFF];
    if (out->autocorr) {
        for (int r = 0; r < 2; ++r)
            for (int k = 0; k < s->n_slots; ++k)
                out->autocorr[r * s->n_slots + k] =
                    s->snap_taken[(size_t)k] ? N - 2 * (int64_t)m[ea::M_AUTO + 2 * k + r] : 0;
        if (out->tw)
            for (int k = 0; k < s->n_slots; ++k) out->tw[k] = s->snap_t[(size_t)k];
    }
    if (out->c4)
        for (int i = 0; i < 3 * (y.R + 1); ++i) out->c4[i] = N - 2 * (int64_t)m[c4_base + i];
    return EA_OK;
}

ea_status ea_c4_shells(ea_sim *s, int32_t n_shells, int64_t *out)
{
    if (!s || !out) return fail(EA_ERR_ARG, "NULL argument");
    const int L = s->lay.L;
    if (L > kMaxShellL) return fail(EA_ERR_ARG, "full-vector C4 is offered for L <= %d (L=%d)", kMaxShellL, L);
    const int max_shells = 3 * (L / 2) * (L / 2) + 1;
    if (n_shells < 1 || n_shells > max_shells)
        return fail(EA_ERR_ARG, "n_shells=%d outside [1, %d]", n_shells, max_shells);
    const int nw = (L + 63) / 64;  // words per row; the doubled row has 2 nw
    const int dw = 2 * nw;
    const size_t q_words = (size_t)L * L * dw;
    if (!s->c4_scratch) {
        hipError_t e = hipMalloc((void **)&s->c4_scratch, 8 * (q_words + (size_t)max_shells));
        if (e != hipSuccess) {
            s->c4_scratch = nullptr;
            return fail(EA_ERR_NOMEM, "hipMalloc(c4 scratch): %s", hipGetErrorString(e));
        }
    }
    unsigned long long *qd = s->c4_scratch, *shells = s->c4_scratch + q_words;
    hipLaunchKernelGGL(ea::zero_u64_kernel, dim3(blocks_for((size_t)n_shells)), dim3(256), 0, s->stream, shells,
                       (size_t)n_shells);
    ea::Geom g = s->geom();
    EA_DISPATCH_W(s->lay.W, hipLaunchKernelGGL((ea::dense_q_kernel<WW>), dim3(blocks_for(q_words)), dim3(256), 0,
                                               s->stream, s->lat, g, dw, qd));
    const bool fft = shells_by_fft(L);
    if (fft) {
        if (!s->fft_work) {
            hipError_t e = hipMalloc(&s->fft_work, fft_work_bytes(L));
            if (e != hipSuccess) {
                s->fft_work = nullptr;
                return fail(EA_ERR_NOMEM, "hipMalloc(c4 FFT work, %zu bytes): %s", fft_work_bytes(L),
                            hipGetErrorString(e));
            }
        }
        ea_status st = launch_fft_shells(qd, dw, L, n_shells, shells, s->fft_work, s->stream);
        if (st != EA_OK) return st;
    } else if (nw <= 2) {
        const dim3 grid((unsigned)((L + ea::kShellRx - 1) / ea::kShellRx), (unsigned)(L * L));
        if (nw == 1)
            hipLaunchKernelGGL((ea::c4_shell_kernel<1>), grid, dim3(256), 0, s->stream, qd, L, n_shells, shells);
        else
            hipLaunchKernelGGL((ea::c4_shell_kernel<2>), grid, dim3(256), 0, s->stream, qd, L, n_shells, shells);
    } else {
        ea_status st = launch_shell_rows(qd, L, n_shells, shells, s->stream);
        if (st != EA_OK) return st;
    }
    EA_HIP(hipGetLastError());
    EA_HIP(hipMemcpyAsync(out, shells, 8 * (size_t)n_shells, hipMemcpyDeviceToHost, s->stream));
    if (fft) return fft_shells_check(s->fft_work, L, s->stream);
    EA_HIP(hipStreamSynchronize(s->stream));
    return EA_OK;
}

ea_status ea_set_shell_route(int32_t route)
{
    if (route != EA_SHELLS_AUTO && route != EA_SHELLS_DIRECT && route != EA_SHELLS_FFT)
        return fail(EA_ERR_ARG, "unknown shell route %d", route);
    g_shell_route.store(route);
    return EA_OK;
}

ea_status ea_get_shell_route(int32_t *route)
{
    if (!route) return fail(EA_ERR_ARG, "NULL argument");
    *route = g_shell_route.load();
    return EA_OK;
}

}  // extern "C"

namespace {

// Scratch of ea_c4_shells_into: the dense q rows of the largest side with
// full-vector C4 (L = 128: 128 x 128 rows of 4 doubled 64-bit words,
// 512 KiB), one array per device for the life of the process.  Host code
// never passes the array's name to a kernel: it passes the device address
// that hipGetSymbolAddress returned for that device.
constexpr size_t kScratchWords =
    (size_t)kMaxShellLNoAlloc * kMaxShellLNoAlloc * 2 * ((kMaxShellLNoAlloc + 63) / 64);
__device__ __align__(256) unsigned long long scratch[kScratchWords];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned long long *g_scratch_ptr[kScratchDevices] = {};  // per device, set on the first call there

// The scratch array's address on `device` (made current by the caller).
ea_status scratch_on(int device, unsigned long long **out)
{
    if (device < 0 || device >= kScratchDevices)
        return fail(EA_ERR_DEVICE, "device %d beyond the %d the library tracks", device, kScratchDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[(size_t)device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(EA_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                        hipGetErrorString(e));
        g_scratch_ptr[(size_t)device] = (unsigned long long *)p;
    }
    *out = g_scratch_ptr[(size_t)device];
    return EA_OK;
}

}  // namespace

extern "C" {

ea_status ea_c4_shells_into(ea_sim *s, int32_t n_shells, int64_t *out_dev)
{
    if (!s || !out_dev) return fail(EA_ERR_ARG, "NULL argument");
    const int L = s->lay.L;
    if (L > kMaxShellLNoAlloc)
        return fail(EA_ERR_ARG, "the allocation-free full-vector C4 is offered for L <= %d (L=%d): the scratch "
                                "array holds the dense overlap of L = %d at most", kMaxShellLNoAlloc, L,
                    kMaxShellLNoAlloc);
    const int max_shells = 3 * (L / 2) * (L / 2) + 1;
    if (n_shells < 1 || n_shells > max_shells)
        return fail(EA_ERR_ARG, "n_shells=%d outside [1, %d]", n_shells, max_shells);
    const int nw = (L + 63) / 64;
    const int dw = 2 * nw;
    const size_t q_words = (size_t)L * L * dw;
    if (q_words > kScratchWords) return fail(EA_ERR_ARG, "L=%d needs %zu scratch words, %zu exist", L, q_words,
                                             kScratchWords);
    int cur = 0;
    EA_HIP(hipGetDevice(&cur));
    if (cur != s->device) EA_HIP(hipSetDevice(s->device));
    unsigned long long *qd = nullptr;
    ea_status st = scratch_on(s->device, &qd);
    if (st == EA_OK) {
        unsigned long long *shells = (unsigned long long *)out_dev;
        hipLaunchKernelGGL(ea::zero_u64_kernel, dim3(blocks_for((size_t)n_shells)), dim3(256), 0, s->stream,
                           shells, (size_t)n_shells);
        ea::Geom g = s->geom();
        switch (s->lay.W) {
#define EA_DENSE_Q(WW)                                                                                         \
    case WW:                                                                                                   \
        hipLaunchKernelGGL((ea::dense_q_kernel<WW>), dim3(blocks_for(q_words)), dim3(256), 0, s->stream, s->lat, \
                           g, dw, qd);                                                                         \
        break;
            EA_DENSE_Q(4) EA_DENSE_Q(8) EA_DENSE_Q(12) EA_DENSE_Q(16) EA_DENSE_Q(20) EA_DENSE_Q(24) EA_DENSE_Q(28)
            EA_DENSE_Q(32)
#undef EA_DENSE_Q
        default: st = fail(EA_ERR_STATE, "unsupported word width %d", s->lay.W);
        }
        if (st == EA_OK) {
            const dim3 grid((unsigned)((L + ea::kShellRx - 1) / ea::kShellRx), (unsigned)(L * L));
            if (nw == 1)
                hipLaunchKernelGGL((ea::c4_shell_kernel<1>), grid, dim3(256), 0, s->stream, qd, L, n_shells, shells);
            else
                hipLaunchKernelGGL((ea::c4_shell_kernel<2>), grid, dim3(256), 0, s->stream, qd, L, n_shells, shells);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) st = fail(EA_ERR_DEVICE, "shell kernels: %s", hipGetErrorString(e));
        }
    }
    if (cur != s->device) {
        const hipError_t e = hipSetDevice(cur);
        if (st == EA_OK && e != hipSuccess) st = fail(EA_ERR_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    }
    return st;
}

ea_status ea_time(const ea_sim *s, uint64_t *t)
{
    if (!s || !t) return fail(EA_ERR_ARG, "NULL argument");
    *t = s->t;
    return EA_OK;
}

ea_status ea_set_time(ea_sim *s, uint64_t t)
{
    if (!s) return fail(EA_ERR_ARG, "sim is NULL");
    if (t >= (1ull << 32)) return fail(EA_ERR_ARG, "t=%llu must be below 2^32", (unsigned long long)t);
    s->t = t;
    return EA_OK;
}

ea_status ea_sync(ea_sim *s)
{
    if (!s) return fail(EA_ERR_ARG, "sim is NULL");
    EA_HIP(hipStreamSynchronize(s->stream));
    return slab_check(s);
}

ea_status ea_set_slab_plan(ea_sim *s, int32_t slabs, int32_t ghost)
{
    if (!s) return fail(EA_ERR_ARG, "sim is NULL");
    if (slabs < -1 || slabs > s->lay.L) return fail(EA_ERR_ARG, "slabs=%d outside [-1, L=%d]", slabs, s->lay.L);
    if (ghost < 0 || ghost > kSlabMaxGhost) return fail(EA_ERR_ARG, "ghost=%d outside [0, %d]", ghost, kSlabMaxGhost);
    if (slabs != -1 && !slab_capable(s->lay.L, s->lay.RW))
        return fail(EA_ERR_ARG, "L=%d with %d words per row cannot run as slabs (a plane of one colour has more "
                                "than %d words)", s->lay.L, s->lay.RW, ea::kSlabThreads);
    const int32_t old_K = s->slab_K, old_g = s->slab_g;
    s->slab_K = slabs;
    s->slab_g = ghost;
    if (slabs > 0) {  // the plan must fit a launch of this run alone
        SlabPlan plan;
        ea_status st = slab_plan_of(s, 1, &plan);
        if (st != EA_OK) {
            s->slab_K = old_K;
            s->slab_g = old_g;
            return st;
        }
    }
    return EA_OK;
}

ea_status ea_get_slab_plan(const ea_sim *s, int32_t *slabs, int32_t *ghost)
{
    if (!s || !slabs || !ghost) return fail(EA_ERR_ARG, "NULL argument");
    SlabPlan plan;
    ea_status st = slab_plan_of(s, 1, &plan);
    if (st != EA_OK) return st;
    *slabs = plan.K > 0 ? plan.K : (plan.K < 0 ? -1 : plan.B / 2);
    *ghost = plan.K < 0 ? 0 : plan.g;
    return EA_OK;
}

// Autotuner of the plain form's packing: for every valid words-per-row of
// side L, a run (p = 0.5, T = 0.8) is timed over a burst of captured sweeps
// after a warm-up; candidates whose final spins differ from the first
// (coarsest) candidate's are rejected, the fastest of the rest is kept for
// the process and appended to the EA_TUNE_CACHE file if that is set.
ea_status ea_tune_plain(int32_t L, int32_t force, int32_t *chosen_rw, ea_tune_choice *tried, int32_t max_tried,
                        int32_t *n_tried)
{
    if (!chosen_rw) return fail(EA_ERR_ARG, "chosen_rw is NULL");
    if (!valid_L(L)) return fail(EA_ERR_ARG, "L=%d must be a multiple of 8 in [8, %d]", L, kMaxL);
    if (n_tried) *n_tried = 0;
    {
        std::lock_guard<std::mutex> lk(g_plain_mu);
        read_plain_tune_file();
        auto it = g_plain_tuned.find(L);
        if (it != g_plain_tuned.end() && !force) {
            *chosen_rw = it->second;
            return EA_OK;
        }
    }
    const int R = L / 2;
    const uint64_t N = (uint64_t)L * L * L;
    uint64_t sweeps = (1ull << 26) / N;
    sweeps = std::max<uint64_t>(64, std::min<uint64_t>(1024, sweeps)) / 64 * 64;
    std::vector<int8_t> ref, cur(2 * (size_t)N);
    int best = 0, n = 0;
    double best_ms = 0.0;
    for (int rw = 1; rw <= R / 4; ++rw) {
        if (!rw_valid(R, rw)) continue;
        ea_config c{};
        c.L = L;
        c.p = 0.5;
        c.T = 0.8;
        c.seed = 7;
        c.words_per_row = rw;
        ea_sim *sim = nullptr;
        ea_status st = ea_create_ex(&c, &sim);
        if (st != EA_OK) return st;
        double ms = 0.0;
        st = ea_sweep(sim, 64);
        if (st == EA_OK) st = ea_sync(sim);
        if (st == EA_OK) {
            const auto t0 = std::chrono::steady_clock::now();
            st = ea_sweep(sim, sweeps);
            if (st == EA_OK) st = ea_sync(sim);
            ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        for (int r = 0; st == EA_OK && r < 2; ++r) st = ea_get_spins(sim, r, cur.data() + (size_t)r * N);
        ea_destroy(sim);
        if (st != EA_OK) return st;
        if (ref.empty()) ref = cur;
        const bool ok = cur == ref;
        if (tried && n < max_tried) {
            tried[n].words_per_row = rw;
            tried[n].threads = 2 * L * L * rw;
            tried[n].select = 1;
            tried[n].ms = ms;
            tried[n].parity_ok = ok ? 1 : 0;
        }
        ++n;
        if (ok && (best == 0 || ms < best_ms)) {
            best = rw;
            best_ms = ms;
        }
    }
    if (n_tried) *n_tried = n;
    *chosen_rw = best;
    std::lock_guard<std::mutex> lk(g_plain_mu);
    g_plain_tuned[L] = best;
    const char *path = std::getenv("EA_TUNE_CACHE");
    if (path && *path) {
        FILE *f = std::fopen(path, "a");
        if (f) {
            std::fprintf(f, "%s plain %d %d %.4f\n", device_arch_name().c_str(), L, best, best_ms);
            std::fclose(f);
        }
    }
    return EA_OK;
}

ea_status ea_get_spins(ea_sim *s, int32_t r, int8_t *pm1)
{
    if (!s || !pm1) return fail(EA_ERR_ARG, "NULL argument");
    if (r < 0 || r > 1) return fail(EA_ERR_ARG, "replica %d not 0 or 1", r);
    const Layout &y = s->lay;
    std::vector<uint32_t> words(2 * (size_t)y.plane);
    EA_HIP(hipMemcpyAsync(words.data(), s->lat.spins + (size_t)r * 2 * y.plane, words.size() * 4,
                          hipMemcpyDeviceToHost, s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));
    ea_status est = slab_check(s);
    if (est != EA_OK) return est;
    const int64_t N = (int64_t)y.L * y.L * y.L;
    for (int64_t i = 0; i < N; ++i) {
        SiteAddr a = address_of(y, i);
        const uint32_t bit = (words[(size_t)a.c * y.plane + a.word] >> a.bit) & 1u;
        pm1[i] = bit ? (int8_t)-1 : (int8_t)1;
    }
    return EA_OK;
}

ea_status ea_set_spins(ea_sim *s, int32_t r, const int8_t *pm1)
{
    if (!s || !pm1) return fail(EA_ERR_ARG, "NULL argument");
    if (r < 0 || r > 1) return fail(EA_ERR_ARG, "replica %d not 0 or 1", r);
    const Layout &y = s->lay;
    const int64_t N = (int64_t)y.L * y.L * y.L;
    std::vector<uint32_t> words(2 * (size_t)y.plane, 0u);
    for (int64_t i = 0; i < N; ++i) {
        if (pm1[i] != 1 && pm1[i] != -1) return fail(EA_ERR_ARG, "spin %lld is %d, not +-1", (long long)i, pm1[i]);
        SiteAddr a = address_of(y, i);
        if (pm1[i] == -1) words[(size_t)a.c * y.plane + a.word] |= 1u << a.bit;
    }
    EA_HIP(hipMemcpyAsync(s->lat.spins + (size_t)r * 2 * y.plane, words.data(), words.size() * 4,
                          hipMemcpyHostToDevice, s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));
    return EA_OK;
}

ea_status ea_get_bonds(ea_sim *s, int8_t *pm1)
{
    if (!s || !pm1) return fail(EA_ERR_ARG, "NULL argument");
    const Layout &y = s->lay;
    std::vector<uint32_t> words(y.bond_words);
    EA_HIP(hipMemcpyAsync(words.data(), s->lat.bonds, words.size() * 4, hipMemcpyDeviceToHost, s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));
    const int64_t N = (int64_t)y.L * y.L * y.L;
    for (int64_t i = 0; i < N; ++i) {
        SiteAddr a = address_of(y, i);
        for (int d = 0; d < 3; ++d) {
            const uint32_t bit = (words[((size_t)d * 2 + a.c) * y.plane + a.word] >> a.bit) & 1u;
            pm1[3 * i + d] = bit ? (int8_t)-1 : (int8_t)1;
        }
    }
    return EA_OK;
}

ea_status ea_set_bonds(ea_sim *s, const int8_t *pm1)
{
    if (!s || !pm1) return fail(EA_ERR_ARG, "NULL argument");
    const Layout &y = s->lay;
    const int64_t N = (int64_t)y.L * y.L * y.L;
    std::vector<uint32_t> words(y.bond_words, 0u);
    for (int64_t i = 0; i < N; ++i) {
        SiteAddr a = address_of(y, i);
        for (int d = 0; d < 3; ++d) {
            const int8_t v = pm1[3 * i + d];
            if (v != 1 && v != -1) return fail(EA_ERR_ARG, "coupling %lld is %d, not +-1", (long long)(3 * i + d), v);
            if (v == -1) words[((size_t)d * 2 + a.c) * y.plane + a.word] |= 1u << a.bit;
        }
    }
    EA_HIP(hipMemcpyAsync(s->lat.bonds, words.data(), words.size() * 4, hipMemcpyHostToDevice, s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));
    return EA_OK;
}

}  // extern "C"

#include "ea_batch_api.h"
#include "ea_server_api.h"
#include "ea_msc_api.h"
#include "ea_shells_api.h"
