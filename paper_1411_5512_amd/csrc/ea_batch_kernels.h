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

// Compile-time geometry of one lattice size.
template <int L>
struct Shape {
    static constexpr int R = L / 2;
    static constexpr int RW = words_per_row_c(R);
    static constexpr int W = R / RW;
    static constexpr int POS = L * L * RW;  // packed words per colour
    static constexpr int NT = POS >= kBatchThreads ? kBatchThreads : ((POS + 63) / 64) * 64;
    static constexpr int P = (POS + NT - 1) / NT;  // words per thread per half-step
    static constexpr int LATTICE_WORDS = 8 * POS;  // 2 spin planes + 6 coupling planes
    static constexpr int LDS_WORDS = LATTICE_WORDS + 16;  // dynamic LDS: lattice + flag
};

// Device-side description of one sample in a batch.
struct BatchJobDev {
    int32_t L;
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

template <int L>
__device__ __forceinline__ uint32_t *lds_spin(int c)
{
    return batch_lds + c * Shape<L>::POS;
}

template <int L>
__device__ __forceinline__ uint32_t *lds_bond(int d, int c)
{
    return batch_lds + (2 + 2 * d + c) * Shape<L>::POS;
}

// Update the colour-c words of this workgroup's replica (eq. 9), reading the
// other colour and the couplings from LDS.
template <int L>
__device__ __forceinline__ void batch_half_step(const BatchJobDev &J, int r, int c, uint32_t t)
{
    using S = Shape<L>;
    constexpr int RW = S::RW, W = S::W;
    uint32_t *own = lds_spin<L>(c);
    const uint32_t *oth = lds_spin<L>(c ^ 1);
    const uint32_t *bx_own = lds_bond<L>(0, c), *by_own = lds_bond<L>(1, c),
                   *bz_own = lds_bond<L>(2, c);
    const uint32_t *bx_oth = lds_bond<L>(0, c ^ 1), *by_oth = lds_bond<L>(1, c ^ 1),
                   *bz_oth = lds_bond<L>(2, c ^ 1);
    const uint32_t c2 = counter_word2(TAG_METRO, (uint32_t)c, (uint32_t)r);
    // Recompute the addresses every half-step: hoisting them out of the
    // sweep loop would keep some thirty address registers live and spill.
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    // one word at a time: a word already carries W/4 independent Philox
    // blocks of instruction-level parallelism, and unrolling further spills
#pragma unroll 1
    for (int k = 0; k < S::P; ++k) {
        const int p = tid + k * S::NT;
        if (S::POS % S::NT != 0 && p >= S::POS) break;
        const int row = p / RW;
        const int w = p - row * RW;
        const int y = row % L;
        const int z = row / L;
        const int par = (y + z + c) & 1;
        const int wm = w == 0 ? RW - 1 : w - 1;
        const int wp = w == RW - 1 ? 0 : w + 1;
        const int ym = (y == 0 ? L - 1 : y - 1) + L * z, yp = (y == L - 1 ? 0 : y + 1) + L * z;
        const int zm = y + L * (z == 0 ? L - 1 : z - 1), zp = y + L * (z == L - 1 ? 0 : z + 1);
        const int base = row * RW;
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
        own[p] = S0 ^ flip_mask_lds<W>(d, t, quad0, c2, J.sample, J.k0, J.k1, batch_tables());
    }
}

// Copy this replica's two colour planes between LDS and a global array.
template <int L>
__device__ __forceinline__ void batch_store_spins(uint32_t *dst)
{
    for (int i = (int)threadIdx.x; i < 2 * Shape<L>::POS; i += Shape<L>::NT) dst[i] = batch_lds[i];
}

// Measurement at time t (index m) of replica r.
template <int L>
__device__ void batch_measure(const BatchJobDev &J, int r, int m, int n_taken)
{
    using S = Shape<L>;
    constexpr int RW = S::RW, W = S::W, POS = S::POS;
    unsigned long long *o = J.obs + (size_t)m * (size_t)J.obs_stride;
    uint32_t unsat = 0, down = 0;
#pragma unroll 1
    for (int c = 0; c < 2; ++c) {
        const uint32_t *own = lds_spin<L>(c);
        const uint32_t *oth = lds_spin<L>(c ^ 1);
        for (int p = (int)threadIdx.x; p < POS; p += S::NT) {
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
            unsat += __popc(Sv ^ xp ^ lds_bond<L>(0, c)[p]) +
                     __popc(xor3(Sv, oth[yp * RW + w], lds_bond<L>(1, c)[p])) +
                     __popc(xor3(Sv, oth[zp * RW + w], lds_bond<L>(2, c)[p]));
            down += __popc(Sv);
        }
    }
    wave_add(o + M_UNSAT + r, unsat);
    wave_add(o + M_DOWN + r, down);
#pragma unroll 1
    for (int k = 0; k < n_taken; ++k) {
        const uint32_t *ref = J.snaps + ((size_t)k * 2 + (size_t)r) * 2 * POS;
        uint32_t diff = 0;
        for (int i = (int)threadIdx.x; i < 2 * POS; i += S::NT) diff += __popc(batch_lds[i] ^ ref[i]);
        wave_add(o + M_AUTO + 2 * k + r, diff);
    }

    // Publish this replica's configuration; the second replica to arrive
    // computes the overlap and C4 from both copies.
    batch_store_spins<L>(J.mspins + ((size_t)m * 2 + (size_t)r) * 2 * POS);
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
    for (int i = (int)threadIdx.x; i < 2 * POS; i += S::NT) qdiff += __popc(q0[i] ^ q1[i]);
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
                for (int p = (int)threadIdx.x; p < POS; p += S::NT) {
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
template <int L>
__device__ void batch_run_unit(const BatchJobDev &J, int r, uint32_t t_stop, bool first)
{
    using S = Shape<L>;
    if ((int)threadIdx.x >= S::NT) return;  // whole surplus waves leave the barrier set
    const uint32_t t0 = J.t_now[r];
    if (!first && t0 >= t_stop) return;
    const uint32_t *src = J.spins + (size_t)r * 2 * S::POS;
    for (int i = (int)threadIdx.x; i < 2 * S::POS; i += S::NT) batch_lds[i] = src[i];
    for (int i = (int)threadIdx.x; i < 6 * S::POS; i += S::NT) batch_lds[2 * S::POS + i] = J.bonds[i];
    fill_select_tables(batch_tables(), J.thr1, J.thr2, J.thr3, (int)threadIdx.x, S::NT);
    __syncthreads();

    int im = 0, iw = 0;
    while (im < J.n_meas && (J.meas_t[im] < t0 || (!first && J.meas_t[im] == t0))) ++im;
    while (iw < J.n_tw && (J.tw_t[iw] < t0 || (!first && J.tw_t[iw] == t0))) ++iw;

    uint32_t t = t0;
    for (;;) {
        if (iw < J.n_tw && J.tw_t[iw] == t) {
            batch_store_spins<L>(J.snaps + ((size_t)iw * 2 + (size_t)r) * 2 * S::POS);
            ++iw;
            __threadfence();
            __syncthreads();
        }
        if (im < J.n_meas && J.meas_t[im] == t) {
            batch_measure<L>(J, r, im, iw);
            ++im;
            __syncthreads();
        }
        if (t >= t_stop) break;
        batch_half_step<L>(J, r, r, t);
        __syncthreads();
        batch_half_step<L>(J, r, r ^ 1, t);
        __syncthreads();
        ++t;
    }
    batch_store_spins<L>(J.spins + (size_t)r * 2 * S::POS);
    if (threadIdx.x == 0) J.t_now[r] = t;
}

__global__ __launch_bounds__(kBatchThreads) void batch_kernel(const BatchJobDev *__restrict__ jobs,
                                                              const BatchUnit *__restrict__ units)
{
    const BatchUnit u = units[blockIdx.x];
    const BatchJobDev J = jobs[u.job];
    switch (J.L) {
    case 8: batch_run_unit<8>(J, u.replica, u.t_stop, u.first != 0); break;
    case 16: batch_run_unit<16>(J, u.replica, u.t_stop, u.first != 0); break;
    case 24: batch_run_unit<24>(J, u.replica, u.t_stop, u.first != 0); break;
    case 32: batch_run_unit<32>(J, u.replica, u.t_stop, u.first != 0); break;
    case 40: batch_run_unit<40>(J, u.replica, u.t_stop, u.first != 0); break;
    case 48: batch_run_unit<48>(J, u.replica, u.t_stop, u.first != 0); break;
    case 56: batch_run_unit<56>(J, u.replica, u.t_stop, u.first != 0); break;
    case 64: batch_run_unit<64>(J, u.replica, u.t_stop, u.first != 0); break;
    default: break;
    }
}

}  // namespace ea
