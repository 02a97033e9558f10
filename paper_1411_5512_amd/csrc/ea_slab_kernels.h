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

// Workgroup b runs slab b mod K of replica (b / K) mod 2 of run b / (2K):
// slab k owns the planes [k L / K, (k + 1) L / K).
struct SlabLaunch {
    SlabRunDev runs[kGroupMax];
    int32_t L, RW, K, g, emax;  // emax: LDS planes per array, at least s + 2 g of every slab
    uint32_t n_half;            // half-steps in this launch (the first is half 0 of sweep t0)
    uint32_t *err;              // set when a wait timed out; every workgroup then ends
};

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

template <int W>
__global__ __launch_bounds__(kSlabThreads) void slab_sweep_kernel(SlabLaunch a)
{
    const int K = a.K, L = a.L, RW = a.RW, PL = L * RW, R = L / 2;
    const int b = (int)blockIdx.x;
    const int slab = b % K, r = (b / K) & 1;
    const SlabRunDev &run = a.runs[b / (2 * K)];
    const int z0 = slab * L / K, s = (slab + 1) * L / K - z0;
    const int g = a.g, E = s + 2 * g, EM = a.emax;
    const int zb = z0 - g;  // global plane of local plane 0, before wrapping
    // LDS: [colour][EM][PL] spins, [direction][colour][EM][PL] couplings, flags
    uint32_t *lspin = slab_lds;
    uint32_t *lbond = slab_lds + 2 * EM * PL;
    uint32_t *flag = slab_lds + 8 * EM * PL;

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

    if (tid == 0) {
        flag[0] = slab_err_seen(a.err);
        flag[1] = 0;
    }
    __syncthreads();
    if (flag[0]) return;

    // the extended region from the state in HBM (the launch boundary makes it whole)
    const size_t plane = (size_t)L * L * RW;
    for (int i = tid; i < E * PL; i += kSlabThreads) {
        const int e = i / PL, c0 = i - e * PL;
        const int zg = wrap(zb + e, L);
        const size_t src = (size_t)zg * PL + c0;
#pragma unroll
        for (int c = 0; c < 2; ++c)
            lspin[(c * EM + e) * PL + c0] = run.spins[((size_t)r * 2 + c) * plane + src];
#pragma unroll
        for (int dc = 0; dc < 6; ++dc) lbond[(dc * EM + e) * PL + c0] = run.bonds[(size_t)dc * plane + src];
    }
    __syncthreads();

    const uint32_t n_half = a.n_half;
    const uint32_t n_cycles = (n_half + (uint32_t)g - 1) / (uint32_t)g;
    const size_t xrep = (size_t)kSlabSlots * 2 * (size_t)L * PL;  // entries per replica
    unsigned long long *xb = run.xbuf + (size_t)r * xrep;
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
            uint32_t *own = lspin + c * EM * PL;
            const uint32_t *oth = lspin + (c ^ 1) * EM * PL;
            const uint32_t *bx_own = lbond + (0 + c) * EM * PL, *by_own = lbond + (2 + c) * EM * PL,
                           *bz_own = lbond + (4 + c) * EM * PL;
            const uint32_t *bx_oth = lbond + (1 - c) * EM * PL, *by_oth = lbond + (3 - c) * EM * PL,
                           *bz_oth = lbond + (5 - c) * EM * PL;
            const int n_items = E - 2 * k;
            if (worker) {
                for (int it = zoff; it < n_items; it += zstep) {
                    const int e = slab_item_plane(it, s, g, k);
                    const int zg = wrap(zb + e, L);
                    const int par = (y + zg + c) & 1;
                    const int base = e * PL;
                    const uint32_t S = own[base + q];
                    const uint32_t O = oth[base + q], Om = oth[base + qm], Op = oth[base + qp];
                    const uint32_t Xo = bx_oth[base + q], Xom = bx_oth[base + qm];
                    const uint32_t Bx = bx_own[base + q], By = by_own[base + q], Bz = bz_own[base + q];
                    const uint32_t Yp = oth[base + qyp], Ym = oth[base + qym], Bym = by_oth[base + qym];
                    const uint32_t Zp = oth[base + PL + q], Zm = oth[base - PL + q], Bzm = bz_oth[base - PL + q];
                    const uint32_t quad0 = (uint32_t)(((y + L * zg) * R + w * W) >> 2);
                    uint32_t uw[W];
                    random_words<W / 4 - 1, W>(t, quad0, c2, run.sample, run.k0, run.k1, uw);
                    const uint32_t pm = 0u - (uint32_t)par;
                    const uint32_t xp = __builtin_amdgcn_bitop3_b32(pm, take_plus1<W>(O, Op), O, kBitopSelect);
                    const uint32_t xm =
                        __builtin_amdgcn_bitop3_b32(pm, O ^ Xo, take_minus1<W>(O ^ Xo, Om ^ Xom), kBitopSelect);
                    const Decision d = classify(S ^ xp ^ Bx, S ^ xm, xor3(S, Yp, By), xor3(S, Ym, Bym),
                                                xor3(S, Zp, Bz), xor3(S, Zm, Bzm));
                    const uint32_t v = S ^ (d.always | accept_words<W / 4 - 1, W>(0u, d, uw, run.thr1, run.thr2,
                                                                                    run.thr3));
                    own[base + q] = v;
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

        // the ghost planes of the next cycle from the owners' publications:
        // both colours, or with g = 1 only the one just updated
        const int nc = g == 1 ? 1 : 2;
        const int c_last = r ^ (int)((j_half - 1) & 1u);
        const int n_ent = 2 * g * nc * PL;
        int bad = 0;
        for (int i0 = tid; i0 < n_ent; i0 += 4 * kSlabThreads) {
            unsigned long long v[4];
            size_t src[4];
            int dst[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int i = i0 + h * kSlabThreads;
                if (i < n_ent) {
                    const int col = i % PL, rest = i / PL;
                    const int cc = nc == 1 ? c_last : (rest & 1);
                    const int gp = rest / nc;  // ghost plane 0 .. 2g-1
                    const int e = gp < g ? gp : s + gp;
                    const int zg = wrap(zb + e, L);
                    src[h] = (((size_t)slot * 2 + cc) * L + zg) * PL + col;
                    dst[h] = (cc * EM + e) * PL + col;
                    v[h] = __hip_atomic_load(xb + src[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int i = i0 + h * kSlabThreads;
                if (i >= n_ent) continue;
                if ((uint32_t)(v[h] >> 32) != epoch) {
                    const unsigned long long start = __builtin_amdgcn_s_memrealtime();
                    for (;;) {
                        __builtin_amdgcn_s_sleep(1);
                        v[h] = __hip_atomic_load(xb + src[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if ((uint32_t)(v[h] >> 32) == epoch) break;
                        if (slab_err_seen(a.err) || __builtin_amdgcn_s_memrealtime() - start > kSlabSpinTicks) {
                            bad = 1;
                            break;
                        }
                    }
                }
                if (bad) break;
                lspin[dst[h]] = (uint32_t)v[h];
            }
            if (bad) break;
        }
        if (bad) {
            __hip_atomic_store(a.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            flag[1] = 1;
        }
        __syncthreads();
        if (flag[1]) return;  // after an error the run's state is undefined
    }

    // the owned planes back to HBM
    for (int i = tid; i < s * PL; i += kSlabThreads) {
        const int e = g + i / PL, c0 = i % PL;
        const size_t dst = (size_t)(z0 + i / PL) * PL + c0;
#pragma unroll
        for (int c = 0; c < 2; ++c) run.spins[((size_t)r * 2 + c) * plane + dst] = lspin[(c * EM + e) * PL + c0];
    }
}

// dst |= src (one word): hands the launch-wide error word to the other runs
// of a group launch without clearing an error they already had.
__global__ void or_word_kernel(uint32_t *dst, const uint32_t *src)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst |= *src;
}

}  // namespace ea
