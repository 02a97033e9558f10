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
    uint32_t *arrive;         // [n_meas] replicas that reached the measurement
    uint32_t *t_now;          // [2] sweeps done per replica
};

// One workgroup's work: replica `replica` of job `job` from its current time
// up to t_stop.
struct BatchUnit {
    int32_t job;
    int32_t replica;
    uint32_t t_stop;
    int32_t first;  // 1 on the job's first span: events at t = 0 are taken too
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
__shared__ uint32_t batch_select_tables[kSelectTableWords];

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

// Update the colour-c words of this workgroup's replica (eq. 9), reading the
// other colour and the couplings from LDS.
template <int L, int RW, int SEL>
__device__ __forceinline__ void batch_half_step(const BatchJobDev &J, int r, int c, uint32_t t)
{
    using S = Shape<L, RW>;
    constexpr int W = S::W;
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
    // one word at a time: a word already carries W/4 independent Philox
    // blocks of instruction-level parallelism, and unrolling further spills
#pragma unroll 1
    for (int p = tid; p < S::POS; p += J.nt) {
        const unsigned row = (unsigned)p / RW;
        const unsigned w = (unsigned)p - row * RW;
        const unsigned y = row % L;
        const unsigned z = row / L;
        const int par = (int)((y + z + (unsigned)c) & 1u);
        const unsigned wm = w == 0 ? RW - 1 : w - 1;
        const unsigned wp = w == RW - 1 ? 0 : w + 1;
        const unsigned ym = (y == 0 ? L - 1 : y - 1) + L * z, yp = (y == L - 1 ? 0 : y + 1) + L * z;
        const unsigned zm = y + L * (z == 0 ? L - 1 : z - 1), zp = y + L * (z == L - 1 ? 0 : z + 1);
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
        const uint32_t a5 = xor3(S0, oth[zp * RW + w], bz_own[p]);
        const uint32_t a6 = xor3(S0, oth[zm * RW + w], bz_oth[zm * RW + w]);
        const Decision d = classify(a1, a2, a3, a4, a5, a6);
        const uint32_t quad0 = (uint32_t)((row * S::R + w * W) >> 2);
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

// Measurement at time t (index m) of replica r.
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

    // Publish this replica's configuration; the second replica to arrive
    // computes the overlap and C4 from both copies.
    batch_store_spins<S>(J.mspins + ((size_t)m * 2 + (size_t)r) * 2 * POS, nt);
    __threadfence();
    __syncthreads();
    uint32_t *flag = batch_lds + S::LATTICE_WORDS;
    if (threadIdx.x == 0) *flag = atomicAdd(J.arrive + m, 1u);
    __syncthreads();
    const bool second = *flag == 1u;
    __syncthreads();
    if (!second) return;
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
        batch_half_step<L, RW, SEL>(J, r, r, t);
        __syncthreads();
        batch_half_step<L, RW, SEL>(J, r, r ^ 1, t);
        __syncthreads();
        ++t;
    }
    batch_store_spins<S>(J.spins + (size_t)r * 2 * S::POS, nt);
    if (threadIdx.x == 0) J.t_now[r] = t;
}

// Dispatch on the packing (finest valid alternative or the default) and the
// select variant for one lattice size.
template <int L>
__device__ __forceinline__ void batch_dispatch_L(const BatchJobDev &J, int r, uint32_t t_stop, bool first)
{
    constexpr int R = L / 2;
    constexpr int RW0 = words_per_row_c(R);
    constexpr int RW1 = finer_words_per_row_c(R, RW0);
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

__global__ __launch_bounds__(kBatchThreads) void batch_kernel(const BatchJobDev *__restrict__ jobs,
                                                              const BatchUnit *__restrict__ units)
{
    const BatchUnit u = units[blockIdx.x];
    const BatchJobDev J = jobs[u.job];
    const bool first = u.first != 0;
    switch (J.L) {
    case 8: batch_dispatch_L<8>(J, u.replica, u.t_stop, first); break;
    case 16: batch_dispatch_L<16>(J, u.replica, u.t_stop, first); break;
    case 24: batch_dispatch_L<24>(J, u.replica, u.t_stop, first); break;
    case 32: batch_dispatch_L<32>(J, u.replica, u.t_stop, first); break;
    case 40: batch_dispatch_L<40>(J, u.replica, u.t_stop, first); break;
    case 48: batch_dispatch_L<48>(J, u.replica, u.t_stop, first); break;
    case 56: batch_dispatch_L<56>(J, u.replica, u.t_stop, first); break;
    case 64: batch_dispatch_L<64>(J, u.replica, u.t_stop, first); break;
    default: break;
    }
}

}  // namespace ea
