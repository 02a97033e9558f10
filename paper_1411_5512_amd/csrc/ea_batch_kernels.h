// ea_batch_kernels.h -- the batched form: one persistent launch runs many
// independent samples of different size, temperature and coupling
// probability.  Each workgroup owns one replica of one sample ("unit") for
// the whole span of sweeps it is given: the replica's spins and the sample's
// couplings sit in LDS, the checkerboard half-steps are separated by
// workgroup barriers instead of kernel launches, and the scheduled snapshots
// and measurements are taken inside the kernel.
//
// The two replicas of a sample never interact, so they run in separate
// workgroups.  Observables of one replica (energy, magnetisation, C(t, t_w))
// are reduced by its own workgroup; the replica-pair observables (overlap and
// C4) need both configurations at the same time t: each workgroup publishes
// its configuration at a measurement time, and whichever arrives second
// computes them from the two published copies.
#pragma once

#include "ea_kernels.h"

namespace ea {

constexpr int kBatchThreads = 1024;
constexpr int kBatchMaxL = 64;
constexpr int kSplitMinL = 48;  // smallest size whose replicas may be split into two z-slabs

__host__ __device__ constexpr int words_per_row_c(int R)
{
    int rw = (R + 31) / 32;
    while ((R / 4) % rw != 0) ++rw;
    return rw;
}

// The next finer valid packing of a row of R sites: the smallest word count
// above rw that splits the row into whole 4-site blocks (0 if none).
__host__ __device__ constexpr int finer_words_per_row_c(int R, int rw)
{
    for (int d = rw + 1; d <= R / 4; ++d)
        if ((R / 4) % d == 0) return d;
    return 0;
}

// Compile-time geometry of one lattice size and row packing.
template <int L, int RW>
struct Shape {
    static constexpr int R = L / 2;
    static constexpr int W = R / RW;
    static constexpr int POS = L * L * RW;  // packed words per colour
    static constexpr int LATTICE_WORDS = 8 * POS;  // 2 spin planes + 6 coupling planes
    static constexpr int LDS_WORDS = LATTICE_WORDS + 16;  // dynamic LDS: lattice + flag
    static_assert(R % RW == 0 && W % 4 == 0 && W <= 32, "invalid row packing");
};

// Threshold select of the update: through the LDS tables or with register
// bit-field selects.
enum : int { SEL_LDS = 0, SEL_REG = 1 };

// Device-side description of one sample in a batch.
struct BatchJobDev {
    int32_t L;
    int32_t rw;   // words per row of the packed layout
    int32_t nt;   // threads of the workgroup that work (multiple of 64, <= kBatchThreads)
    int32_t sel;  // SEL_LDS or SEL_REG
    uint32_t k0, k1, sample;
    uint32_t thr1, thr2, thr3;
    int32_t n_meas, n_tw, obs_stride;
    uint32_t *spins;          // [replica][colour][POS]: state between launches
    const uint32_t *bonds;    // [direction][colour][POS]
    uint32_t *snaps;          // [slot][replica][colour][POS]
    uint32_t *mspins;         // [measurement][replica][colour][POS]
    const uint32_t *meas_t;   // [n_meas], strictly increasing
    const uint32_t *tw_t;     // [n_tw], strictly increasing
    unsigned long long *obs;  // [n_meas][obs_stride]
    uint32_t *arrive;         // [n_meas] workgroups that reached the measurement
    uint32_t *t_now;          // [2] sweeps done per replica
    int32_t parts;            // workgroups per replica: 1, or 2 for a replica split into z-slabs
    uint32_t *xbuf;           // split: [replica][slab][sweep parity][colour][first/last plane][L * rw]
    unsigned long long *pub;  // split: [replica][slab] boundary publications (see batch_run_split)
    uint32_t *err;            // set when a split pair gave up waiting for its partner
};

// One workgroup's work: replica `replica` of job `job` from its current time
// up to t_stop.
struct BatchUnit {
    int32_t job;
    int32_t replica;
    uint32_t t_stop;
    int32_t first;  // 1 on the job's first span: events at t = 0 are taken too
    int32_t slab;   // split jobs: which z-slab (0 or 1); 0 otherwise
};

// Observable slots of one measurement (popcounts, like the plain form):
// [0,1] unsatisfied bonds, [2,3] spins down, [4] S_0 != S_1,
// [5 + 2k + r] S_r(t) != S_r(tw_k), then [5 + 2 n_tw + d (R+1) + rho] for C4.
__device__ __forceinline__ int batch_c4_base(int n_tw) { return M_AUTO + 2 * n_tw; }

// The workgroup's LDS: the threshold-select tables are a static array (its
// address is a compile-time constant, so table reads need no address add),
// followed by the dynamic part: [colour][POS] spins of the replica,
// [direction][colour][POS] couplings and one word for a broadcast flag.
// Declared at file scope so that every access is a plain ds_read/ds_write.
extern __shared__ uint32_t batch_lds[];
__shared__ __align__(16) uint32_t batch_select_tables[kSelectTableWords];

__device__ __forceinline__ uint32_t *batch_tables() { return batch_select_tables; }

template <class S>
__device__ __forceinline__ uint32_t *lds_spin(int c)
{
    return batch_lds + c * S::POS;
}

template <class S>
__device__ __forceinline__ uint32_t *lds_bond(int d, int c)
{
    return batch_lds + (2 + 2 * d + c) * S::POS;
}

// Update the colour-C words of this workgroup's replica (eq. 9), reading the
// other colour and the couplings from LDS.  The colour is a template
// argument so that every plane's LDS offset is a compile-time constant.
template <int L, int RW, int SEL, int C>
__device__ __forceinline__ void batch_half_step(const BatchJobDev &J, int r, uint32_t t)
{
    using S = Shape<L, RW>;
    constexpr int W = S::W;
    constexpr int c = C;
    uint32_t *own = lds_spin<S>(c);
    const uint32_t *oth = lds_spin<S>(c ^ 1);
    const uint32_t *bx_own = lds_bond<S>(0, c), *by_own = lds_bond<S>(1, c), *bz_own = lds_bond<S>(2, c);
    const uint32_t *bx_oth = lds_bond<S>(0, c ^ 1), *by_oth = lds_bond<S>(1, c ^ 1),
                   *bz_oth = lds_bond<S>(2, c ^ 1);
    const uint32_t c2 = counter_word2(TAG_METRO, (uint32_t)c, (uint32_t)r);
    // Recompute the addresses every half-step: hoisting them out of the
    // sweep loop would keep some thirty address registers live and spill.
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    // Each thread keeps one (y, w) column of the z-planes and walks z in
    // steps of nt / PLANE (threads past the last whole column stay idle), so
    // the y and x neighbour offsets are computed once per half-step.  One
    // word at a time: a word already carries W/4 independent Philox blocks of
    // instruction-level parallelism, and unrolling further spills.
    constexpr unsigned PLANE = (unsigned)(L * RW);
    const unsigned q = (unsigned)tid % PLANE;
    const unsigned w = q % RW;
    const unsigned y = q / RW;
    const unsigned dz = (unsigned)J.nt / PLANE;
    const unsigned z_first = (unsigned)tid < dz * PLANE ? (unsigned)tid / PLANE : (unsigned)L;
    const unsigned qm = q - w + (w == 0 ? RW - 1 : w - 1);  // word w - 1 of the row (cyclic)
    const unsigned qp = q - w + (w == RW - 1 ? 0 : w + 1);  // word w + 1
    const unsigned qym = (y == 0 ? L - 1 : y - 1) * RW + w;
    const unsigned qyp = (y == L - 1 ? 0 : y + 1) * RW + w;
    const unsigned par0 = (y + (unsigned)c) & 1u;
    const unsigned quad_col = (y * S::R + w * W) >> 2;  // y R + w W is a multiple of 4
#pragma unroll 1
    for (unsigned z = z_first; z < (unsigned)L; z += dz) {
        const unsigned base = z * PLANE;
        const unsigned p = base + q;
        const int par = (int)((par0 ^ z) & 1u);
        const unsigned zm = (z == 0 ? L - 1 : z - 1) * PLANE + q, zp = (z == L - 1 ? 0 : z + 1) * PLANE + q;
        const uint32_t S0 = own[p];
        const uint32_t O = oth[p], Om = oth[base + qm], Op = oth[base + qp];
        const uint32_t Xo = bx_oth[p], Xom = bx_oth[base + qm];
        const uint32_t xp = par ? take_plus1<W>(O, Op) : O;
        const uint32_t xm = par ? (O ^ Xo) : take_minus1<W>(O ^ Xo, Om ^ Xom);
        const uint32_t a1 = S0 ^ xp ^ bx_own[p];
        const uint32_t a2 = S0 ^ xm;
        const uint32_t a3 = xor3(S0, oth[base + qyp], by_own[p]);
        const uint32_t a4 = xor3(S0, oth[base + qym], by_oth[base + qym]);
        const uint32_t a5 = xor3(S0, oth[zp], bz_own[p]);
        const uint32_t a6 = xor3(S0, oth[zm], bz_oth[zm]);
        const Decision d = classify(a1, a2, a3, a4, a5, a6);
        const uint32_t quad0 = quad_col + ((z * (unsigned)(L * S::R)) >> 2);  // (row R + w W) / 4, row = y + L z
        uint32_t flips;
        if constexpr (SEL == SEL_LDS)
            flips = flip_mask_lds<W>(d, t, quad0, c2, J.sample, J.k0, J.k1, batch_tables());
        else
            flips = flip_mask<W>(d, t, quad0, c2, J.sample, J.k0, J.k1, J.thr1, J.thr2, J.thr3);
        own[p] = S0 ^ flips;
    }
}

// Copy this replica's two colour planes between LDS and a global array.
template <class S>
__device__ __forceinline__ void batch_store_spins(uint32_t *dst, int nt)
{
    for (int i = (int)threadIdx.x; i < 2 * S::POS; i += nt) dst[i] = batch_lds[i];
}

// Publish this workgroup's part of replica r's configuration at measurement
// m (rows [row0, row0 + rows) of both colours, taken from LDS spin words
// batch_lds[c * src_stride + i]); the last workgroup of the job to arrive
// computes the replica-pair observables, the overlap and C4 (eqs. 2, 3), from
// the published copies.  flag_word is a free LDS word for a broadcast.
template <int L, int RW>
__device__ void batch_publish_and_pair(const BatchJobDev &J, int r, int m, int row0, int rows, int src_stride,
                                       int flag_word)
{
    using S = Shape<L, RW>;
    constexpr int W = S::W, POS = S::POS;
    const int nt = J.nt;
    unsigned long long *o = J.obs + (size_t)m * (size_t)J.obs_stride;
    uint32_t *dst = J.mspins + ((size_t)m * 2 + (size_t)r) * 2 * POS;
    const int n = rows * RW;
#pragma unroll 1
    for (int c = 0; c < 2; ++c)
        for (int i = (int)threadIdx.x; i < n; i += nt) dst[c * POS + row0 * RW + i] = batch_lds[c * src_stride + i];
    __threadfence();
    __syncthreads();
    uint32_t *flag = batch_lds + flag_word;
    if (threadIdx.x == 0) *flag = atomicAdd(J.arrive + m, 1u);
    __syncthreads();
    const bool last = *flag == (uint32_t)(2 * J.parts - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();

    const uint32_t *q0 = J.mspins + (size_t)m * 4 * POS;
    const uint32_t *q1 = q0 + 2 * POS;
    uint32_t qdiff = 0;
    for (int i = (int)threadIdx.x; i < 2 * POS; i += nt) qdiff += __popc(q0[i] ^ q1[i]);
    wave_add(o + M_QDIFF, qdiff);

    unsigned long long *c4 = o + batch_c4_base(J.n_tw);
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
#pragma unroll 1
        for (int rho = 0; rho <= S::R; ++rho) {
            uint32_t diff = 0;
#pragma unroll 1
            for (int c = 0; c < 2; ++c) {
                const int cp = c ^ (rho & 1);
#pragma unroll 1
                for (int p = (int)threadIdx.x; p < POS; p += nt) {
                    const int row = p / RW;
                    const int w = p - row * RW;
                    const int y = row % L;
                    const int z = row / L;
                    const uint32_t q = q0[c * POS + p] ^ q1[c * POS + p];
                    uint32_t qp;
                    if (d == 0) {
                        const int par = (y + z + c) & 1;
                        const int kx = (rho & 1) ? (rho - 1) / 2 + par : rho / 2;
                        const int start = (w * W + kx) % S::R;
                        const int wi = start / W;
                        const int off = start - wi * W;
                        const int wj = wi + 1 == RW ? 0 : wi + 1;
                        const uint32_t lo = q0[cp * POS + row * RW + wi] ^ q1[cp * POS + row * RW + wi];
                        const uint32_t hi = q0[cp * POS + row * RW + wj] ^ q1[cp * POS + row * RW + wj];
                        qp = off == 0 ? lo : (((lo >> off) | (hi << (W - off))) & word_mask<W>());
                    } else {
                        const int prow = d == 1 ? (y + rho) % L + L * z : y + L * ((z + rho) % L);
                        qp = q0[cp * POS + prow * RW + w] ^ q1[cp * POS + prow * RW + w];
                    }
                    diff += __popc(q ^ qp);
                }
            }
            wave_add(c4 + d * (S::R + 1) + rho, diff);
        }
    }
}

// Measurement at time t (index m) of replica r (whole replica in LDS).
template <int L, int RW>
__device__ void batch_measure(const BatchJobDev &J, int r, int m, int n_taken)
{
    using S = Shape<L, RW>;
    constexpr int W = S::W, POS = S::POS;
    const int nt = J.nt;
    unsigned long long *o = J.obs + (size_t)m * (size_t)J.obs_stride;
    uint32_t unsat = 0, down = 0;
#pragma unroll 1
    for (int c = 0; c < 2; ++c) {
        const uint32_t *own = lds_spin<S>(c);
        const uint32_t *oth = lds_spin<S>(c ^ 1);
        for (int p = (int)threadIdx.x; p < POS; p += nt) {
            const int row = p / RW;
            const int w = p - row * RW;
            const int y = row % L;
            const int z = row / L;
            const int par = (y + z + c) & 1;
            const int wp = w == RW - 1 ? 0 : w + 1;
            const int yp = (y == L - 1 ? 0 : y + 1) + L * z;
            const int zp = y + L * (z == L - 1 ? 0 : z + 1);
            const uint32_t Sv = own[p];
            const uint32_t O = oth[row * RW + w];
            const uint32_t xp = par ? take_plus1<W>(O, oth[row * RW + wp]) : O;
            unsat += __popc(Sv ^ xp ^ lds_bond<S>(0, c)[p]) +
                     __popc(xor3(Sv, oth[yp * RW + w], lds_bond<S>(1, c)[p])) +
                     __popc(xor3(Sv, oth[zp * RW + w], lds_bond<S>(2, c)[p]));
            down += __popc(Sv);
        }
    }
    wave_add(o + M_UNSAT + r, unsat);
    wave_add(o + M_DOWN + r, down);
#pragma unroll 1
    for (int k = 0; k < n_taken; ++k) {
        const uint32_t *ref = J.snaps + ((size_t)k * 2 + (size_t)r) * 2 * POS;
        uint32_t diff = 0;
        for (int i = (int)threadIdx.x; i < 2 * POS; i += nt) diff += __popc(batch_lds[i] ^ ref[i]);
        wave_add(o + M_AUTO + 2 * k + r, diff);
    }
    batch_publish_and_pair<L, RW>(J, r, m, 0, L * L, POS, S::LATTICE_WORDS);
}

// Run one unit: load the replica and the couplings into LDS, sweep up to
// t_stop taking the events scheduled in (t0, t_stop] (and at t0 itself on the
// job's first span), then write the replica back.
template <int L, int RW, int SEL>
__device__ void batch_run_unit(const BatchJobDev &J, int r, uint32_t t_stop, bool first)
{
    using S = Shape<L, RW>;
    const int nt = J.nt;
    if ((int)threadIdx.x >= nt) return;  // whole surplus waves leave the barrier set
    const uint32_t t0 = J.t_now[r];
    if (!first && t0 >= t_stop) return;
    const uint32_t *src = J.spins + (size_t)r * 2 * S::POS;
    for (int i = (int)threadIdx.x; i < 2 * S::POS; i += nt) batch_lds[i] = src[i];
    for (int i = (int)threadIdx.x; i < 6 * S::POS; i += nt) batch_lds[2 * S::POS + i] = J.bonds[i];
    if constexpr (SEL == SEL_LDS) fill_select_tables(batch_tables(), J.thr1, J.thr2, J.thr3, (int)threadIdx.x, nt);
    __syncthreads();

    int im = 0, iw = 0;
    while (im < J.n_meas && (J.meas_t[im] < t0 || (!first && J.meas_t[im] == t0))) ++im;
    while (iw < J.n_tw && (J.tw_t[iw] < t0 || (!first && J.tw_t[iw] == t0))) ++iw;

    uint32_t t = t0;
    for (;;) {
        if (iw < J.n_tw && J.tw_t[iw] == t) {
            batch_store_spins<S>(J.snaps + ((size_t)iw * 2 + (size_t)r) * 2 * S::POS, nt);
            ++iw;
            __threadfence();
            __syncthreads();
        }
        if (im < J.n_meas && J.meas_t[im] == t) {
            batch_measure<L, RW>(J, r, im, iw);
            ++im;
            __syncthreads();
        }
        if (t >= t_stop) break;
        if (r == 0) {
            batch_half_step<L, RW, SEL, 0>(J, r, t);
            __syncthreads();
            batch_half_step<L, RW, SEL, 1>(J, r, t);
        } else {
            batch_half_step<L, RW, SEL, 1>(J, r, t);
            __syncthreads();
            batch_half_step<L, RW, SEL, 0>(J, r, t);
        }
        __syncthreads();
        ++t;
    }
    batch_store_spins<S>(J.spins + (size_t)r * 2 * S::POS, nt);
    if (threadIdx.x == 0) J.t_now[r] = t;
}

// ---------------------------------------------------------------------------
// Split replicas.  In a batch of uneven sizes one replica of the largest
// sample on one CU sets the length of the launch.  Such a replica can instead
// be cut into two z-slabs of NZ = L/2 planes, each held in LDS by its own
// workgroup.  A site on a slab's first or last plane has one neighbour on the
// other slab's adjacent plane (periodic in z), of the other colour; those
// boundary words pass through a small exchange area in global memory.
//
// In each half-step wave 0 updates the slab's two boundary planes: it waits
// until the partner slab has published its boundary words of the previous
// half-step (a counter stored with release, read with acquire, agent scope),
// updates its own boundary words and publishes them.  The other waves update
// the interior planes meanwhile, which need nothing from the partner, so the
// exchange latency hides behind interior work; the half-step still ends with
// one workgroup barrier.  Publication counter of a slab: 1 once its state at
// t = 0 is out, 2t + h + 2 after half-step h of sweep t.  Boundary words
// written in sweep t go to slot t & 1 (the state at t = 0 to slot 1): a
// measurement at t reads both colours of the partner's slot (t - 1) & 1
// while the partner may already be writing sweep t into the other slot.  A wait gives up
// after kSplitSpinTicks of the 100 MHz real-time counter (20 s), flags J.err
// and ends the unit, so a launch always drains.

constexpr unsigned long long kSplitSpinTicks = 2000000000ull;

template <int L, int RW>
struct Slab {
    static constexpr int R = L / 2, W = R / RW;
    static constexpr int NZ = L / 2;            // planes per slab
    static constexpr int PL = L * RW;           // words of one plane of one colour
    static constexpr int SPOS = NZ * PL;        // slab words of one colour
    static constexpr int POS = L * L * RW;      // whole-lattice words of one colour
    static constexpr int HALO = 8 * SPOS;       // [colour][PL] z couplings of the plane below the slab
    static constexpr int FLAG = HALO + 2 * PL;  // broadcast words
    static constexpr int LDS_WORDS = FLAG + 16;
    static_assert(NZ >= 3 && R % RW == 0 && W % 4 == 0 && W <= 32, "invalid slab");
};

template <class S>
__device__ __forceinline__ uint32_t *slab_spin(int c)
{
    return batch_lds + c * S::SPOS;
}

template <class S>
__device__ __forceinline__ uint32_t *slab_bond(int d, int c)
{
    return batch_lds + (2 + 2 * d + c) * S::SPOS;
}

// Boundary words of (replica r, slab, slot, colour c, plane k: 0 first, 1 last).
template <class S>
__device__ __forceinline__ uint32_t *slab_xbuf(const BatchJobDev &J, int r, int slab, int slot, int c, int k)
{
    return J.xbuf +
           (((((size_t)r * 2 + (size_t)slab) * 2 + (size_t)slot) * 2 + (size_t)c) * 2 + (size_t)k) * S::PL;
}

__device__ __forceinline__ uint32_t load_agent(const uint32_t *p)
{
    return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave 0: wait until the counter reaches `want`; false on time-out.
__device__ __forceinline__ bool slab_wait(unsigned long long *pub, unsigned long long want)
{
    int ok = 1;
    if (threadIdx.x == 0) {
        const unsigned long long start = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(pub, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < want) {
            __builtin_amdgcn_s_sleep(1);
            if (__builtin_amdgcn_s_memrealtime() - start > kSplitSpinTicks) {
                ok = 0;
                break;
            }
        }
    }
    ok = __shfl(ok, 0, 64);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok != 0;
}

// Wave 0: make this wave's boundary stores visible, then set the counter.
__device__ __forceinline__ void slab_publish(unsigned long long *pub, unsigned long long value)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (threadIdx.x == 0) __hip_atomic_store(pub, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// The half-step exchange without cache maintenance.  The boundary words go
// out with agent-scope stores, which are written through to the level shared
// by all XCDs, and the partner reads them with agent-scope loads, which do
// not hit a stale L2 line; so publishing only has to wait for this wave's
// stores to complete before the counter is set, and waiting only has to see
// the counter -- no L2 write-back or invalidation per half-step.
__device__ __forceinline__ void store_agent(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void slab_publish_words(unsigned long long *pub, unsigned long long value)
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (threadIdx.x == 0) __hip_atomic_store(pub, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool slab_wait_words(unsigned long long *pub, unsigned long long want)
{
    int ok = 1;
    if (threadIdx.x == 0) {
        const unsigned long long start = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
            __builtin_amdgcn_s_sleep(1);
            if (__builtin_amdgcn_s_memrealtime() - start > kSplitSpinTicks) {
                ok = 0;
                break;
            }
        }
    }
    ok = __shfl(ok, 0, 64);
    asm volatile("" ::: "memory");
    return ok != 0;
}

// New value of slab word p (colour c, sweep t), given its z-1 and z+1
// neighbour words of the other colour and the coupling to the z-1 neighbour.
template <int L, int RW, int SEL>
__device__ __forceinline__ uint32_t slab_new_word(const BatchJobDev &J, int r, int c, uint32_t t, int z0, int p,
                                                  uint32_t Ozm, uint32_t Ozp, uint32_t Bzm)
{
    using S = Slab<L, RW>;
    constexpr int W = S::W;
    const uint32_t *own = slab_spin<S>(c);
    const uint32_t *oth = slab_spin<S>(c ^ 1);
    const uint32_t *bx_own = slab_bond<S>(0, c), *by_own = slab_bond<S>(1, c), *bz_own = slab_bond<S>(2, c);
    const uint32_t *bx_oth = slab_bond<S>(0, c ^ 1), *by_oth = slab_bond<S>(1, c ^ 1);
    const unsigned row = (unsigned)p / RW;  // slab row y + L zl
    const unsigned w = (unsigned)p - row * RW;
    const unsigned y = row % L;
    const unsigned zl = row / L;
    const int par = (int)((y + zl + (unsigned)z0 + (unsigned)c) & 1u);
    const unsigned wm = w == 0 ? RW - 1 : w - 1;
    const unsigned wp = w == RW - 1 ? 0 : w + 1;
    const unsigned ym = (y == 0 ? L - 1 : y - 1) + L * zl, yp = (y == L - 1 ? 0 : y + 1) + L * zl;
    const unsigned base = row * RW;
    const uint32_t S0 = own[p];
    const uint32_t O = oth[base + w], Om = oth[base + wm], Op = oth[base + wp];
    const uint32_t Xo = bx_oth[base + w], Xom = bx_oth[base + wm];
    const uint32_t xp = par ? take_plus1<W>(O, Op) : O;
    const uint32_t xm = par ? (O ^ Xo) : take_minus1<W>(O ^ Xo, Om ^ Xom);
    const uint32_t a1 = S0 ^ xp ^ bx_own[p];
    const uint32_t a2 = S0 ^ xm;
    const uint32_t a3 = xor3(S0, oth[yp * RW + w], by_own[p]);
    const uint32_t a4 = xor3(S0, oth[ym * RW + w], by_oth[ym * RW + w]);
    const uint32_t a5 = xor3(S0, Ozp, bz_own[p]);
    const uint32_t a6 = xor3(S0, Ozm, Bzm);
    const Decision d = classify(a1, a2, a3, a4, a5, a6);
    const uint32_t quad0 = (uint32_t)(((row + (unsigned)(L * z0)) * S::R + w * W) >> 2);
    const uint32_t c2 = counter_word2(TAG_METRO, (uint32_t)c, (uint32_t)r);
    uint32_t flips;
    if constexpr (SEL == SEL_LDS)
        flips = flip_mask_lds<W>(d, t, quad0, c2, J.sample, J.k0, J.k1, batch_tables());
    else
        flips = flip_mask<W>(d, t, quad0, c2, J.sample, J.k0, J.k1, J.thr1, J.thr2, J.thr3);
    return S0 ^ flips;
}

// Half-step (t, colour c) of one slab.  Returns false (wave 0 only) if the
// partner never published.
template <int L, int RW, int SEL>
__device__ __forceinline__ bool slab_half_step(const BatchJobDev &J, int r, int slab, int c, uint32_t t,
                                               unsigned long long want, unsigned long long done)
{
    using S = Slab<L, RW>;
    const int z0 = slab * S::NZ;
    uint32_t *own = slab_spin<S>(c);
    const uint32_t *oth = slab_spin<S>(c ^ 1);
    const uint32_t *bz_oth = slab_bond<S>(2, c ^ 1);
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (tid >= 64) {
        // interior planes 1 .. NZ-2
#pragma unroll 1
        for (int p = S::PL + tid - 64; p < S::SPOS - S::PL; p += J.nt - 64)
            own[p] = slab_new_word<L, RW, SEL>(J, r, c, t, z0, p, oth[p - S::PL], oth[p + S::PL], bz_oth[p - S::PL]);
        return true;
    }
    if (!slab_wait_words(J.pub + 2 * r + (slab ^ 1), want)) return false;
    // colour c ^ 1 was last written in the previous half-step: this sweep's
    // first half-step, or the previous sweep's second
    const int rslot = (int)((c == r ? t + 1 : t) & 1u);
    const int wslot = (int)(t & 1u);
    const uint32_t *part_last = slab_xbuf<S>(J, r, slab ^ 1, rslot, c ^ 1, 1);   // the plane below this slab
    const uint32_t *part_first = slab_xbuf<S>(J, r, slab ^ 1, rslot, c ^ 1, 0);  // the plane above it
    const uint32_t *halo_bz = batch_lds + S::HALO + (c ^ 1) * S::PL;
#pragma unroll 1
    for (int i = tid; i < 2 * S::PL; i += 64) {
        const int k = i >= S::PL ? 1 : 0;
        const int j = i - k * S::PL;
        const int p = k ? S::SPOS - S::PL + j : j;
        uint32_t v;
        if (k == 0)
            v = slab_new_word<L, RW, SEL>(J, r, c, t, z0, p, load_agent(part_last + j), oth[p + S::PL], halo_bz[j]);
        else
            v = slab_new_word<L, RW, SEL>(J, r, c, t, z0, p, oth[p - S::PL], load_agent(part_first + j),
                                          bz_oth[p - S::PL]);
        own[p] = v;
        store_agent(slab_xbuf<S>(J, r, slab, wslot, c, k) + j, v);
    }
    slab_publish_words(J.pub + 2 * r + slab, done);
    return true;
}

// Measurement m at time t of one slab: its partial sums, then its part of
// the published configuration.  The partner's first plane (the +z neighbour
// of this slab's last plane) comes from the exchange area; wave 0 has waited
// for the partner's state at t.
template <int L, int RW>
__device__ void slab_measure(const BatchJobDev &J, int r, int slab, int m, int n_taken, uint32_t t)
{
    using S = Slab<L, RW>;
    constexpr int W = S::W;
    const int nt = J.nt;
    const int z0 = slab * S::NZ;
    unsigned long long *o = J.obs + (size_t)m * (size_t)J.obs_stride;
    uint32_t unsat = 0, down = 0;
#pragma unroll 1
    for (int c = 0; c < 2; ++c) {
        const uint32_t *own = slab_spin<S>(c);
        const uint32_t *oth = slab_spin<S>(c ^ 1);
        const uint32_t *part_first = slab_xbuf<S>(J, r, slab ^ 1, (int)((t + 1) & 1u), c ^ 1, 0);
        for (int p = (int)threadIdx.x; p < S::SPOS; p += nt) {
            const int row = p / RW;
            const int w = p - row * RW;
            const int y = row % L;
            const int zl = row / L;
            const int par = (y + zl + z0 + c) & 1;
            const int wp = w == RW - 1 ? 0 : w + 1;
            const int yp = (y == L - 1 ? 0 : y + 1) + L * zl;
            const uint32_t Sv = own[p];
            const uint32_t O = oth[row * RW + w];
            const uint32_t xp = par ? take_plus1<W>(O, oth[row * RW + wp]) : O;
            const uint32_t Ozp = zl + 1 < S::NZ ? oth[p + S::PL] : load_agent(part_first + (p - (S::SPOS - S::PL)));
            unsat += __popc(Sv ^ xp ^ slab_bond<S>(0, c)[p]) +
                     __popc(xor3(Sv, oth[yp * RW + w], slab_bond<S>(1, c)[p])) +
                     __popc(xor3(Sv, Ozp, slab_bond<S>(2, c)[p]));
            down += __popc(Sv);
        }
    }
    wave_add(o + M_UNSAT + r, unsat);
    wave_add(o + M_DOWN + r, down);
#pragma unroll 1
    for (int k = 0; k < n_taken; ++k) {
        const uint32_t *ref = J.snaps + ((size_t)k * 2 + (size_t)r) * 2 * S::POS + (size_t)z0 * S::PL;
        uint32_t diff = 0;
#pragma unroll 1
        for (int c = 0; c < 2; ++c)
            for (int i = (int)threadIdx.x; i < S::SPOS; i += nt) diff += __popc(batch_lds[c * S::SPOS + i] ^ ref[c * S::POS + i]);
        wave_add(o + M_AUTO + 2 * k + r, diff);
    }
    batch_publish_and_pair<L, RW>(J, r, m, z0 * L, S::NZ * L, S::SPOS, S::FLAG);
}

// Copy this slab's two colour parts between LDS and a [colour][POS] array.
template <class S>
__device__ __forceinline__ void slab_store(uint32_t *dst, int z0, int nt)
{
#pragma unroll 1
    for (int c = 0; c < 2; ++c)
        for (int i = (int)threadIdx.x; i < S::SPOS; i += nt)
            dst[(size_t)c * S::POS + (size_t)z0 * S::PL + i] = batch_lds[c * S::SPOS + i];
}

// Run one slab of a split replica up to t_stop (events as in batch_run_unit).
template <int L, int RW, int SEL>
__device__ void batch_run_slab(const BatchJobDev &J, int r, int slab, uint32_t t_stop, bool first)
{
    using S = Slab<L, RW>;
    const int nt = J.nt;
    if ((int)threadIdx.x >= nt) return;
    const uint32_t t0 = J.t_now[r];
    if (!first && t0 >= t_stop) return;
    const int z0 = slab * S::NZ;
    const int zb = (z0 + L - 1) % L;  // the plane below the slab
    const uint32_t *src = J.spins + (size_t)r * 2 * S::POS;
    for (int c = 0; c < 2; ++c)
        for (int i = (int)threadIdx.x; i < S::SPOS; i += nt)
            batch_lds[c * S::SPOS + i] = src[(size_t)c * S::POS + (size_t)z0 * S::PL + i];
    for (int dc = 0; dc < 6; ++dc)
        for (int i = (int)threadIdx.x; i < S::SPOS; i += nt)
            batch_lds[(2 + dc) * S::SPOS + i] = J.bonds[(size_t)dc * S::POS + (size_t)z0 * S::PL + i];
    for (int c = 0; c < 2; ++c)
        for (int i = (int)threadIdx.x; i < S::PL; i += nt)
            batch_lds[S::HALO + c * S::PL + i] = J.bonds[(size_t)(4 + c) * S::POS + (size_t)zb * S::PL + i];
    if constexpr (SEL == SEL_LDS) fill_select_tables(batch_tables(), J.thr1, J.thr2, J.thr3, (int)threadIdx.x, nt);
    uint32_t *abort_flag = batch_lds + S::FLAG + 1;
    if (threadIdx.x == 0) *abort_flag = 0;
    __syncthreads();
    unsigned long long *my_pub = J.pub + 2 * r + slab;
    if (first && threadIdx.x < 64) {
        // the state at t = 0 of both colours' boundary planes
        for (int c = 0; c < 2; ++c)
            for (int i = (int)threadIdx.x; i < 2 * S::PL; i += 64) {
                const int k = i >= S::PL ? 1 : 0;
                const int j = i - k * S::PL;
                slab_xbuf<S>(J, r, slab, 1, c, k)[j] = batch_lds[c * S::SPOS + (k ? S::SPOS - S::PL : 0) + j];
            }
        slab_publish(my_pub, 1ull);
    }

    int im = 0, iw = 0;
    while (im < J.n_meas && (J.meas_t[im] < t0 || (!first && J.meas_t[im] == t0))) ++im;
    while (iw < J.n_tw && (J.tw_t[iw] < t0 || (!first && J.tw_t[iw] == t0))) ++iw;

    uint32_t t = t0;
    for (;;) {
        if (iw < J.n_tw && J.tw_t[iw] == t) {
            slab_store<S>(J.snaps + ((size_t)iw * 2 + (size_t)r) * 2 * S::POS, z0, nt);
            ++iw;
            __threadfence();
            __syncthreads();
        }
        if (im < J.n_meas && J.meas_t[im] == t) {
            if (threadIdx.x < 64 && !slab_wait(J.pub + 2 * r + (slab ^ 1), 2ull * t + 1)) {
                if (threadIdx.x == 0) {
                    *abort_flag = 1;
                    atomicOr(J.err, 1u);
                }
            }
            __syncthreads();
            if (*abort_flag) return;
            slab_measure<L, RW>(J, r, slab, im, iw, t);
            ++im;
            __syncthreads();
        }
        if (t >= t_stop) break;
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            const unsigned long long want = 2ull * t + (unsigned)h + 1, done = want + 1;
            if (!slab_half_step<L, RW, SEL>(J, r, slab, r ^ h, t, want, done) && threadIdx.x == 0) {
                *abort_flag = 1;
                atomicOr(J.err, 1u);
            }
            __syncthreads();
            if (*abort_flag) return;
        }
        ++t;
    }
    slab_store<S>(J.spins + (size_t)r * 2 * S::POS, z0, nt);
    if (threadIdx.x == 0) J.t_now[r] = t;
}

// Dispatch on the packing (finest valid alternative or the default) and the
// select variant for one lattice size.
template <int L>
__device__ __forceinline__ void batch_dispatch_L(const BatchJobDev &J, int r, int slab, uint32_t t_stop, bool first)
{
    constexpr int R = L / 2;
    constexpr int RW0 = words_per_row_c(R);
    constexpr int RW1 = finer_words_per_row_c(R, RW0);
    if constexpr (L >= kSplitMinL) {
        if (J.parts == 2) {
            if (J.rw == RW0 && J.sel == SEL_LDS) batch_run_slab<L, RW0, SEL_LDS>(J, r, slab, t_stop, first);
            return;
        }
    }
    if (J.rw == RW0) {
        if (J.sel == SEL_LDS) batch_run_unit<L, RW0, SEL_LDS>(J, r, t_stop, first);
        else batch_run_unit<L, RW0, SEL_REG>(J, r, t_stop, first);
    } else if constexpr (RW1 != 0) {
        if (J.rw == RW1) {
            if (J.sel == SEL_LDS) batch_run_unit<L, RW1, SEL_LDS>(J, r, t_stop, first);
            else batch_run_unit<L, RW1, SEL_REG>(J, r, t_stop, first);
        }
    }
}

// poison, lds_words: the debug LDS fill (debug_poison; poison = 0: off) of
// the launch's dynamic LDS words and the select tables.
__global__ __launch_bounds__(kBatchThreads) void batch_kernel(const BatchJobDev *__restrict__ jobs,
                                                              const BatchUnit *__restrict__ units,
                                                              uint32_t poison, int lds_words)
{
    if (poison) {
        debug_poison(batch_lds, lds_words, poison, (int)threadIdx.x, kBatchThreads);
        debug_poison(batch_select_tables, kSelectTableWords, poison, (int)threadIdx.x, kBatchThreads);
        __syncthreads();
    }
    const BatchUnit u = units[blockIdx.x];
    const BatchJobDev J = jobs[u.job];
    const bool first = u.first != 0;
    switch (J.L) {
    case 8: batch_dispatch_L<8>(J, u.replica, u.slab, u.t_stop, first); break;
    case 16: batch_dispatch_L<16>(J, u.replica, u.slab, u.t_stop, first); break;
    case 24: batch_dispatch_L<24>(J, u.replica, u.slab, u.t_stop, first); break;
    case 32: batch_dispatch_L<32>(J, u.replica, u.slab, u.t_stop, first); break;
    case 40: batch_dispatch_L<40>(J, u.replica, u.slab, u.t_stop, first); break;
    case 48: batch_dispatch_L<48>(J, u.replica, u.slab, u.t_stop, first); break;
    case 56: batch_dispatch_L<56>(J, u.replica, u.slab, u.t_stop, first); break;
    case 64: batch_dispatch_L<64>(J, u.replica, u.slab, u.t_stop, first); break;
    default: break;
    }
}

}  // namespace ea
