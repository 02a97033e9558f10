// ea_slab_kernels.h -- the plain form's persistent path: one launch runs many
// sweeps of one or more runs of one geometry, each replica cut into z-slabs
// that stay in LDS for the whole launch.
//
// The paper synchronises the whole lattice with one kernel call per
// checkerboard half-step (Sec. III).  Here every replica is cut into K slabs
// of consecutive z-planes; a workgroup holds its slab's s planes plus g
// ghost planes on either side (spins of both colours and all six coupling
// planes) in LDS and runs g half-steps in a row on that extended region: a
// half-step updates colour c on a plane from colour 1 - c on the plane and
// its two z neighbours, so the planes that are still correct shrink by one
// on each side per half-step, and after g half-steps exactly the owned
// planes are.  The random word of a site depends only on (seed, sample,
// replica, sweep, site) (reading 7), so the ghost planes are updated
// redundantly to the very same values their owner computes, and the result
// is bit-identical to one launch per half-step.  Then the slabs exchange:
// each publishes its owned planes that lie within g planes of a face, both
// colours, and reads the 2g ghost planes of the next cycle from its
// neighbours' publications.  With g = 1 the ghost planes keep the colour
// that was not updated, and only the updated colour moves.
//
// Exchange entries are 64-bit words {spin word, epoch << 32}, stored and
// loaded at agent scope (through the level that all XCDs share): a reader
// polls each entry until its epoch is the one it waits for, so data and
// signal travel together and no flag, fence or cache maintenance is needed.
// Publications of cycle m go to slot m mod 3 of [slot][colour][z][plane
// word], so a slot is rewritten only after every reader has passed the cycle
// that read it.  Epochs count cycles from a per-run serial the host advances
// after every launch, so an entry left by an earlier launch never matches.
//
// Every wait gives up after kSlabSpinTicks of the 100 MHz real-time counter,
// sets the error word and ends the workgroup; waiting workgroups watch the
// error word and end too, so a launch always drains.
#pragma once

#include "ea_kernels.h"

namespace ea {

constexpr int kSlabThreads = 1024;
constexpr int kSlabSlots = 3;
constexpr unsigned long long kSlabSpinTicks = 1000000000ull;  // 10 s

// One run of a slab launch (all runs of a launch share L, the packing, the
// slab plan and g).
struct SlabRunDev {
    uint32_t *spins;          // [replica][colour][plane]: state before and after the launch
    const uint32_t *bonds;    // [direction][colour][plane]
    unsigned long long *xbuf; // [replica][slot][colour][L planes][PL] exchange entries
    uint32_t k0, k1, sample, thr1, thr2, thr3;
    uint32_t t0;              // sweep index of the launch's first half-step
    uint32_t serial;          // epoch of cycle m is serial + m + 1
};

// The replicas of a launch laid end to end (replica q = 2 run + r, its
// plane z at index q L + z, P = 2 L runs planes in all); workgroup b owns the
// planes [b P / B, (b + 1) P / B): one slab of one replica, or the end of one
// replica and the start of the next (B >= 2 runs keeps a share within L
// planes).  With B = 2 runs K this is K slabs per replica, slab k owning the
// planes [k L / K, (k + 1) L / K).
struct SlabLaunch {
    SlabRunDev runs[kGroupMax];
    int32_t L, RW, g;
    int32_t B, P;        // workgroups, planes of all replicas
    int32_t emax;        // LDS planes per array: the extended regions of a workgroup's pieces
    int32_t tables;      // 2: a workgroup's second piece (another run) has its own select table
    uint32_t n_half;     // half-steps in this launch (the first is half 0 of sweep t0)
    uint32_t *err;       // set when a wait timed out; every workgroup then ends
    uint32_t order;      // debug order of the shares (debug_block); 0 = workgroup b takes share b
    uint32_t poison;     // debug LDS fill before the loads (debug_poison); 0 = off
};

// One piece of a workgroup's share: owned planes [z0, z0 + s) of replica r
// of run `run`, its extended region (g ghost planes either side) at local
// LDS planes [off, off + s + 2 g).
struct SlabPiece {
    int run, r, z0, s, off;
};

__device__ __forceinline__ int slab_pieces(const SlabLaunch &a, int b, SlabPiece &p0, SlabPiece &p1)
{
    const int L = a.L;
    const int start = (int)((long long)b * a.P / a.B), end = (int)((long long)(b + 1) * a.P / a.B);
    const int q0 = start / L, cut = (q0 + 1) * L;
    p0.run = q0 >> 1;
    p0.r = q0 & 1;
    p0.z0 = start - q0 * L;
    p0.s = min(end, cut) - start;
    p0.off = 0;
    p1 = p0;
    if (end <= cut) return 1;
    p1.run = (q0 + 1) >> 1;
    p1.r = (q0 + 1) & 1;
    p1.z0 = 0;
    p1.s = end - cut;
    p1.off = p0.s + 2 * a.g;
    return 2;
}

extern __shared__ uint32_t slab_lds[];

__device__ __forceinline__ uint32_t slab_err_seen(uint32_t *err)
{
    return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Local plane of work item j of the half-step that updates the planes
// [k, E - k) of the extended region: the owned planes [g, g + s) first,
// alternately from the two faces inwards (so that the planes the neighbours
// wait for are done first), then the ghost planes below and above.
__device__ __forceinline__ int slab_item_plane(int j, int s, int g, int k)
{
    if (j < s) return g + ((j & 1) ? s - 1 - (j >> 1) : (j >> 1));
    j -= s;
    const int lo = g - k;
    return j < lo ? k + j : g + s + (j - lo);
}

// Acceptance bits of a word's W sites from their random words u and their
// thresholds thr (bit i set iff u[i] < thr[i]), built from the top block
// down as in accept_words.
template <int J, int W>
__device__ __forceinline__ uint32_t below_each(uint32_t accept, const uint32_t (&u)[W], const uint32_t (&thr)[W])
{
    accept = append_below4(accept, u[4 * J + 3], thr[4 * J + 3], u[4 * J + 2], thr[4 * J + 2], u[4 * J + 1],
                           thr[4 * J + 1], u[4 * J], thr[4 * J]);
    if constexpr (J > 0)
        return below_each<J - 1, W>(accept, u, thr);
    else
        return accept;
}

// The general acceptance of a word with thresholds from the LDS select
// table (fill_select_tables): four sites per 16-byte read, as in
// flip_mask_lds, but with the random words already drawn.
template <int W>
__device__ __forceinline__ uint32_t accept_words_tab(const Decision &d, const uint32_t (&u)[W], const uint32_t *tab)
{
    uint32_t thr[W];
    select_thresholds<W>(d, tab, thr);
    return below_each<W / 4 - 1, W>(0u, u, thr);
}

// accept_screened with the general case through the tables: where uphill
// moves of dE >= 8 are rare, a word none of whose random words falls below
// thr2 accepts exactly its n = 2 sites whose word is below thr1; other words
// take the table select, so the decisions are the same either way.
template <int W, bool SCREEN>
__device__ __forceinline__ uint32_t accept_slab(const Decision &d, const uint32_t (&u)[W], uint32_t thr1,
                                                uint32_t thr2, uint32_t thr3, const uint32_t *tab)
{
    if constexpr (SCREEN) {
        const bool rare = (uint64_t)thr2 * (uint64_t)W < (1ull << 24) && thr3 <= thr2;  // uniform
        if (rare) {
            const uint32_t a1 = below_words<W / 4 - 1, W>(0u, u, thr1);
            uint32_t v[W];
#pragma unroll
            for (int i = 0; i < W; ++i) v[i] = u[i];
#pragma unroll
            for (int n = W; n > 1; n = (n + 2) / 3) {
#pragma unroll
                for (int i = 0; 3 * i < n; ++i) {
                    uint32_t m = v[3 * i];
                    if (3 * i + 1 < n) m = min(m, v[3 * i + 1]);
                    if (3 * i + 2 < n) m = min(m, v[3 * i + 2]);
                    v[i] = m;
                }
            }
            if (v[0] >= thr2) return a1 & d.any & ~d.always;
        }
    }
    return accept_words_tab<W>(d, u, tab);
}

// The LDS planes a half-step of colour c reads and writes.
struct SlabPlanes {
    uint32_t *own;
    const uint32_t *oth, *bx_own, *by_own, *bz_own, *bx_oth, *by_oth, *bz_oth;
};

__device__ __forceinline__ SlabPlanes slab_planes(uint32_t *lspin, const uint32_t *lbond, int stride, int c)
{
    SlabPlanes P;
    P.own = lspin + c * stride;
    P.oth = lspin + (c ^ 1) * stride;
    P.bx_own = lbond + (0 + c) * stride;
    P.by_own = lbond + (2 + c) * stride;
    P.bz_own = lbond + (4 + c) * stride;
    P.bx_oth = lbond + (1 - c) * stride;
    P.by_oth = lbond + (3 - c) * stride;
    P.bz_oth = lbond + (5 - c) * stride;
    return P;
}

// One packed word's update (eq. 9): its own word and the fifteen words
// around it, the W random words, and the flip decision.  Zm and Zp (the z
// neighbours of the other colour) may be replaced before update() by words
// that come from a neighbouring slab.
template <int W>
struct SlabWord {
    uint32_t S, O, Om, Op, Xo, Xom, Bx, By, Bz, Yp, Ym, Bym, Zp, Zm, Bzm;
    uint32_t u[W];

    __device__ __forceinline__ void load(const SlabPlanes &P, int base, int q, int qm, int qp, int qym, int qyp,
                                         int PL)
    {
        S = P.own[base + q];
        O = P.oth[base + q];
        Om = P.oth[base + qm];
        Op = P.oth[base + qp];
        Xo = P.bx_oth[base + q];
        Xom = P.bx_oth[base + qm];
        Bx = P.bx_own[base + q];
        By = P.by_own[base + q];
        Bz = P.bz_own[base + q];
        Yp = P.oth[base + qyp];
        Ym = P.oth[base + qym];
        Bym = P.by_oth[base + qym];
        Zp = P.oth[base + PL + q];
        Zm = P.oth[base - PL + q];
        Bzm = P.bz_oth[base - PL + q];
    }

    __device__ __forceinline__ void draw(uint32_t t, uint32_t quad0, uint32_t c2, uint32_t sample, uint32_t k0,
                                         uint32_t k1)
    {
        random_words<W / 4 - 1, W>(t, quad0, c2, sample, k0, k1, u);
    }

    // par: the row's x parity (x = 2 xh + par)
    template <bool SCREEN>
    __device__ __forceinline__ uint32_t update(int par, uint32_t thr1, uint32_t thr2, uint32_t thr3,
                                               const uint32_t *tab) const
    {
        const uint32_t pm = 0u - (uint32_t)par;
        const uint32_t xp = __builtin_amdgcn_bitop3_b32(pm, take_plus1<W>(O, Op), O, kBitopSelect);
        const uint32_t xm = __builtin_amdgcn_bitop3_b32(pm, O ^ Xo, take_minus1<W>(O ^ Xo, Om ^ Xom), kBitopSelect);
        const Decision d = classify(S ^ xp ^ Bx, S ^ xm, xor3(S, Yp, By), xor3(S, Ym, Bym), xor3(S, Zp, Bz),
                                    xor3(S, Zm, Bzm));
        return S ^ (d.always | accept_slab<W, SCREEN>(d, u, thr1, thr2, thr3, tab));
    }
};

// Wait until the entry at p carries `epoch` (it did not on a first look);
// false if the error word is set or the wait times out.
__device__ __forceinline__ bool slab_poll(const unsigned long long *p, uint32_t epoch, uint32_t *err,
                                          unsigned long long &v)
{
    const unsigned long long start = __builtin_amdgcn_s_memrealtime();
    for (;;) {
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(const_cast<unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 32) == epoch) return true;
        if (slab_err_seen(err) || __builtin_amdgcn_s_memrealtime() - start > kSlabSpinTicks) return false;
    }
}

__shared__ __align__(16) uint32_t slab_select_tables[kSelectTableWords];

// SCREEN: launches whose slabs give every SIMD four or more waves of work
// per half-step screen the rare uphill moves (accept_slab); smaller ones are
// bound by one wave's chain of dependent instructions, which the screen
// lengthens.  SPAN: some workgroup's share spans two replicas (two pieces);
// launches of whole slabs take the one-piece instantiation, whose constants
// all stay in scalar registers across the half-steps.
template <int W, bool SCREEN, bool SPAN>
__global__ __launch_bounds__(kSlabThreads) void slab_sweep_kernel(SlabLaunch a)
{
    const int L = a.L, RW = a.RW, PL = L * RW, R = L / 2;
    const int g = a.g, EM = a.emax;
    // consecutive shares (z neighbours) on the same XCD, whose exchange is
    // faster than one across XCDs (xcd_block); the debug order permutes first
    SlabPiece p0, p1;
    const int share = xcd_block(debug_block((int)blockIdx.x, (int)gridDim.x, a.order), (int)gridDim.x);
    const int np = slab_pieces(a, share, p0, p1);
    // LDS: [colour][EM][PL] spins, [direction][colour][EM][PL] couplings,
    // 16 flag words, then (tables = 2) the second piece's select table
    uint32_t *lspin = slab_lds;
    uint32_t *lbond = slab_lds + 2 * EM * PL;
    uint32_t *flag = slab_lds + 8 * EM * PL;
    uint32_t *tab1 = flag + 16;

    // threads: column q of the z-planes, plane offset zoff, zstep planes at once
    const int zstep = kSlabThreads / PL;
    const int tid = (int)threadIdx.x;
    const bool worker = tid < zstep * PL;
    const int q = tid % PL, zoff = tid / PL;
    const int w = q % RW, y = q / RW;
    const int qm = q - w + (w == 0 ? RW - 1 : w - 1);
    const int qp = q - w + (w == RW - 1 ? 0 : w + 1);
    const int qym = (y == 0 ? L - 1 : y - 1) * RW + w;
    const int qyp = (y == L - 1 ? 0 : y + 1) * RW + w;

    if (a.poison) {
        debug_poison(slab_lds, 8 * EM * PL + 16 + (a.tables == 2 ? kSelectTableWords : 0), a.poison, tid,
                     kSlabThreads);
        debug_poison(slab_select_tables, kSelectTableWords, a.poison, tid, kSlabThreads);
        __syncthreads();
    }
    if (tid == 0) {
        flag[0] = slab_err_seen(a.err);
        flag[1] = 0;
    }
    __syncthreads();
    if (flag[0]) return;
    if (np > 1 && (g > 1 || !SPAN)) {  // the host plans two-piece shares for SPAN launches at depth 1 only
        if (tid == 0) __hip_atomic_store(a.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }

    // the extended regions from the state in HBM (the launch boundary makes them whole)
    const size_t plane = (size_t)L * L * RW;
    for (int pi = 0; pi < np; ++pi) {
        const SlabPiece pc = pi ? p1 : p0;
        const SlabRunDev &run = a.runs[pc.run];
        const int E = pc.s + 2 * g, zb = pc.z0 - g;
        for (int i = tid; i < E * PL; i += kSlabThreads) {
            const int e = i / PL, c0 = i - e * PL;
            const int le = pc.off + e;
            const size_t src = (size_t)wrap(zb + e, L) * PL + c0;
#pragma unroll
            for (int c = 0; c < 2; ++c)
                lspin[(c * EM + le) * PL + c0] = run.spins[((size_t)pc.r * 2 + c) * plane + src];
#pragma unroll
            for (int dc = 0; dc < 6; ++dc) lbond[(dc * EM + le) * PL + c0] = run.bonds[(size_t)dc * plane + src];
        }
    }
    const SlabRunDev &run0 = a.runs[p0.run];
    const SlabRunDev &run1 = a.runs[p1.run];
    fill_select_tables(slab_select_tables, run0.thr1, run0.thr2, run0.thr3, tid, kSlabThreads);
    if (a.tables == 2 && np > 1) fill_select_tables(tab1, run1.thr1, run1.thr2, run1.thr3, tid, kSlabThreads);
    __syncthreads();

    const uint32_t n_half = a.n_half;
    const size_t xrep = (size_t)kSlabSlots * 2 * (size_t)L * PL;  // entries per replica

    if (g == 1) {
        // One half-step per exchange.  A boundary word's only neighbour outside
        // its piece is its z neighbour in the ghost plane, same column, of the
        // colour the neighbouring slab updated in the previous half-step: the
        // thread that updates the word loads that entry itself before its
        // random words and checks the epoch after them, so no ghost pass and
        // no extra barrier are needed, and the interior planes overlap the
        // exchange.  Ghost planes in LDS are read only in the first half-step.
        // (Measured: a look after the random words instead, or a second look
        // there, is 5-10% slower at L = 64.)
        const uint32_t *tab_1 = a.tables == 2 ? tab1 : slab_select_tables;
        for (uint32_t j = 0; j < n_half; ++j) {
            const int slot_now = (int)(j % (uint32_t)kSlabSlots);
            const int slot_prev = (int)((j + (uint32_t)kSlabSlots - 1u) % (uint32_t)kSlabSlots);
            // the pieces one after the other, each with its constants uniform
            // across the workgroup; a thread's items continue its stride
            // (items zoff, zoff + zstep, ... over both pieces' planes)
#pragma unroll
            for (int pi = 0; pi < (SPAN ? 2 : 1); ++pi) {
                if (pi >= np) break;
                const SlabPiece pc = pi ? p1 : p0;
                const SlabRunDev &run = pi ? run1 : run0;
                const uint32_t *tab = pi ? tab_1 : slab_select_tables;
                const int s = pc.s, z0 = pc.z0, r = pc.r, off = pc.off;
                const int first = pi ? p0.s : 0;  // item number of the piece's first plane
                const int c = r ^ (int)(j & 1u);
                const uint32_t t = run.t0 + (j >> 1);
                const uint32_t ep_prev = run.serial + j, ep_now = run.serial + j + 1u;
                const uint32_t c2 = counter_word2(TAG_METRO, (uint32_t)c, (uint32_t)r);
                unsigned long long *xb = run.xbuf + (size_t)r * xrep;
                unsigned long long *gl = xb + (((size_t)slot_prev * 2 + (c ^ 1)) * L + wrap(z0 - 1, L)) * PL + q;
                unsigned long long *gu = xb + (((size_t)slot_prev * 2 + (c ^ 1)) * L + wrap(z0 + s, L)) * PL + q;
                unsigned long long *pub = xb + ((size_t)slot_now * 2 + c) * (size_t)L * PL + q;
                const SlabPlanes P = slab_planes(lspin, lbond, EM * PL, c);
                if (!worker) continue;
                int it = zoff;
                if (first > it) it += ((first - it + zstep - 1) / zstep) * zstep;
                for (; it < first + s; it += zstep) {
                    const int jj = it - first;
                    const int e = 1 + ((jj & 1) ? s - 1 - (jj >> 1) : (jj >> 1));
                    const bool lo = e == 1, hi = e == s;
                    const bool need_lo = lo && j > 0, need_hi = hi && j > 0;
                    const int zg = z0 + e - 1;
                    // the ghost words are loaded first, so that their latency
                    // overlaps the LDS loads and the random words
                    unsigned long long vl = 0, vu = 0;
                    if (need_lo) vl = __hip_atomic_load(gl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (need_hi) vu = __hip_atomic_load(gu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const int base = (off + e) * PL;
                    SlabWord<W> sw;
                    sw.load(P, base, q, qm, qp, qym, qyp, PL);
                    __builtin_amdgcn_sched_barrier(0);
                    sw.draw(t, (uint32_t)(((y + L * zg) * R + w * W) >> 2), c2, run.sample, run.k0, run.k1);
                    if (need_lo && (uint32_t)(vl >> 32) != ep_prev && !slab_poll(gl, ep_prev, a.err, vl)) flag[1] = 1;
                    if (need_hi && (uint32_t)(vu >> 32) != ep_prev && !slab_poll(gu, ep_prev, a.err, vu)) flag[1] = 1;
                    if (need_lo) sw.Zm = (uint32_t)vl;
                    if (need_hi) sw.Zp = (uint32_t)vu;
                    const uint32_t v = sw.template update<SCREEN>((y + zg + c) & 1, run.thr1, run.thr2, run.thr3, tab);
                    P.own[base + q] = v;
                    if (lo || hi)
                        __hip_atomic_store(pub + (size_t)zg * PL, ((unsigned long long)ep_now << 32) | v,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            __syncthreads();
            if (flag[1]) {
                if (tid == 0) __hip_atomic_store(a.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;  // after an error the run's state is undefined
            }
        }
    } else {
        // g half-steps per exchange on the shrinking extended region of the
        // workgroup's one slab, then the 2g ghost planes (both colours) from
        // the owners' publications.
        const SlabRunDev &run = run0;
        const int r = p0.r, z0 = p0.z0, s = p0.s, E = s + 2 * g, zb = z0 - g;
        unsigned long long *xb = run.xbuf + (size_t)r * xrep;
        const uint32_t *tab = slab_select_tables;
        const uint32_t n_cycles = (n_half + (uint32_t)g - 1) / (uint32_t)g;
        uint32_t j_half = 0;
        for (uint32_t m = 0; m < n_cycles; ++m) {
            const int G = (int)min((uint32_t)g, n_half - m * (uint32_t)g);
            const uint32_t epoch = run.serial + m + 1u;
            const int slot = (int)(m % (uint32_t)kSlabSlots);
            for (int k = 1; k <= G; ++k, ++j_half) {
                const uint32_t t = run.t0 + (j_half >> 1);
                const int c = r ^ (int)(j_half & 1u);
                const bool publish = k >= G - 1;  // the colour's last update in this cycle
                const uint32_t c2 = counter_word2(TAG_METRO, (uint32_t)c, (uint32_t)r);
                const SlabPlanes P = slab_planes(lspin, lbond, EM * PL, c);
                const int n_items = E - 2 * k;
                if (worker) {
                    for (int it = zoff; it < n_items; it += zstep) {
                        const int e = slab_item_plane(it, s, g, k);
                        const int zg = wrap(zb + e, L);
                        SlabWord<W> sw;
                        sw.load(P, e * PL, q, qm, qp, qym, qyp, PL);
                        sw.draw(t, (uint32_t)(((y + L * zg) * R + w * W) >> 2), c2, run.sample, run.k0, run.k1);
                        const uint32_t v =
                            sw.template update<SCREEN>((y + zg + c) & 1, run.thr1, run.thr2, run.thr3, tab);
                        P.own[e * PL + q] = v;
                        // owned planes within g of a face are read by the neighbours
                        if (publish && it < s && (e - g < g || g + s - 1 - e < g))
                            __hip_atomic_store(xb + (((size_t)slot * 2 + c) * L + zg) * PL + q,
                                               ((unsigned long long)epoch << 32) | v, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                __syncthreads();
            }
            if (m + 1 == n_cycles) break;

            // the ghost planes of the next cycle, both colours: each thread's
            // entries, up to eight at a time, all re-read together until their
            // epochs match
            const int n_ent = 2 * g * 2 * PL;
            bool ok = true;
            for (int i0 = tid; ok && i0 < n_ent; i0 += 8 * kSlabThreads) {
                unsigned long long *src[8];
                int dst[8];
                uint32_t pend = 0;
#pragma unroll
                for (int h = 0; h < 8; ++h) {
                    const int i = i0 + h * kSlabThreads;
                    src[h] = xb;
                    dst[h] = 0;
                    if (i < n_ent) {
                        const int col = i % PL, rest = i / PL;
                        const int cc = rest & 1, gp = rest >> 1;  // ghost plane 0 .. 2g-1
                        const int e = gp < g ? gp : s + gp;
                        src[h] = xb + (((size_t)slot * 2 + cc) * L + wrap(zb + e, L)) * PL + col;
                        dst[h] = (cc * EM + e) * PL + col;
                        pend |= 1u << h;
                    }
                }
                const unsigned long long start = __builtin_amdgcn_s_memrealtime();
                for (;;) {
                    unsigned long long v[8];
#pragma unroll
                    for (int h = 0; h < 8; ++h)
                        if ((pend >> h) & 1u) v[h] = __hip_atomic_load(src[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                    for (int h = 0; h < 8; ++h)
                        if (((pend >> h) & 1u) && (uint32_t)(v[h] >> 32) == epoch) {
                            lspin[dst[h]] = (uint32_t)v[h];
                            pend &= ~(1u << h);
                        }
                    if (!pend) break;
                    if (slab_err_seen(a.err) || __builtin_amdgcn_s_memrealtime() - start > kSlabSpinTicks) {
                        ok = false;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            if (!ok) {
                __hip_atomic_store(a.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                flag[1] = 1;
            }
            __syncthreads();
            if (flag[1]) return;  // after an error the run's state is undefined
        }
    }

    // the owned planes back to HBM
    for (int pi = 0; pi < np; ++pi) {
        const SlabPiece pc = pi ? p1 : p0;
        const SlabRunDev &run = a.runs[pc.run];
        for (int i = tid; i < pc.s * PL; i += kSlabThreads) {
            const int e = pc.off + g + i / PL, c0 = i % PL;
            const size_t dst = (size_t)(pc.z0 + i / PL) * PL + c0;
#pragma unroll
            for (int c = 0; c < 2; ++c)
                run.spins[((size_t)pc.r * 2 + c) * plane + dst] = lspin[(c * EM + e) * PL + c0];
        }
    }
}

// dst |= src (one word): hands the launch-wide error word to the other runs
// of a group launch without clearing an error they already had.
__global__ void or_word_kernel(uint32_t *dst, const uint32_t *src)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst |= *src;
}

}  // namespace ea
