// ea_msc_kernels.h -- asynchronous multispin coding (Sec. III): the same site
// of several samples sits in the bits of one 32-bit word, and one random word
// per (sweep, colour, replica, site) serves every sample of the word.
//
// Multispin layout.  A batch holds B samples; one word carries M = min(B, 32)
// of them and G = B / M word sets (G = 2 for B = 64) share the random words.
// With M < 32 a word carries S = 32 / M sites of each sample: the lattice is
// cut along z into S slabs of Lz = L / S planes (Lz even), and bit k M + m of
// the word at reduced position (x, y, z') holds sample m at z = z' + k Lz
// (the slab split of Sec. III).  A z-neighbour across a slab face sits in the
// word at the other face of the reduced lattice, rotated by M bits.  Colours
// follow the reduced coordinates, (x + y + z') & 1, equal to the full site's
// colour because Lz is even.  Each (word set, replica, colour) plane holds
// P = R L Lz words (R = L/2), word index xh + R (y + L z'), xh = x >> 1.
// Spins and couplings carry 1 for -1, as in the one-sample layout; the
// couplings to +x, +y, +z live in three planes per colour, like the spins.
#pragma once

#include "ea_device.h"

namespace ea {

constexpr uint32_t TAG_SHARED = 3u;  // counter tag of the shared Metropolis words

// Division by a run-time constant d <= 2^16 of x < 2^24: q = (x m) >> 40 with
// m = floor(2^40 / d) + 1 is exact, since x d < 2^40 keeps the rounding error
// of m below one step of x / d.
struct Divider {
    uint64_t m;
    __device__ __forceinline__ uint32_t div(uint32_t x) const { return (uint32_t)(((uint64_t)x * m) >> 40); }
};

struct MscGeom {
    int L, R, Lz;
    int P;   // words per plane
    int q;   // threads per plane: four consecutive xh each
    Divider by_r4, by_l;  // divisions by R / 4 and by L
    uint32_t order = 0;   // debug order of the half-step launch's blocks (debug_block)
};

struct MscLattice {
    uint32_t *spins;  // [G][replica 2][colour 2][P]
    uint32_t *bonds;  // [G][direction 3][colour 2][P]
};

__device__ __forceinline__ size_t msc_spin_plane(const MscGeom &g, int gi, int r, int c)
{
    return (((size_t)gi * 2 + (size_t)r) * 2 + (size_t)c) * (size_t)g.P;
}

__device__ __forceinline__ size_t msc_bond_plane(const MscGeom &g, int gi, int d, int c)
{
    return (((size_t)gi * 3 + (size_t)d) * 2 + (size_t)c) * (size_t)g.P;
}

// The word of the slab above aligned to this one: bit k M + m takes bit
// (k + 1) M + m, slab S - 1 takes slab 0 (the periodic face).
template <int M>
__device__ __forceinline__ uint32_t from_slab_above(uint32_t w)
{
    if constexpr (M == 32)
        return w;
    else
        return (w >> M) | (w << (32 - M));
}

// The word of the slab below aligned to this one: bit k M + m takes bit
// (k - 1) M + m.
template <int M>
__device__ __forceinline__ uint32_t from_slab_below(uint32_t w)
{
    if constexpr (M == 32)
        return w;
    else
        return (w << M) | (w >> (32 - M));
}

// Shift by n slabs up (n >= 0): bit k M + m takes bit (k + n) M + m.
template <int M>
__device__ __forceinline__ uint32_t from_slabs_above(uint32_t w, int n)
{
    if constexpr (M == 32) {
        return w;
    } else {
        const int s = (n * M) & 31;
        return s ? (w >> s) | (w << (32 - s)) : w;
    }
}

__device__ __forceinline__ uint4 load4(const uint32_t *p)
{
    return *reinterpret_cast<const uint4 *>(p);
}

// Loads at a 32-bit word offset from a wave-uniform plane base.  (Forming
// the byte offset in 32 bits, which lets the compiler use scalar-base
// addressing, measured 2-4% slower here.)
__device__ __forceinline__ uint4 load4_at(const uint32_t *base, uint32_t word)
{
    return *reinterpret_cast<const uint4 *>(base + word);
}

__device__ __forceinline__ uint32_t load_at(const uint32_t *base, uint32_t word)
{
    return base[word];
}

// --------------------------------------------------------------------------
// Couplings and initial spins (Sec. II), sample by sample with the keys of
// the one-sample form: sample sample0 + gi M + m draws, for the full site h,
// the words the one-sample form draws for it.  One thread per four
// consecutive xh of a row; grid.y = what (0..2 coupling direction, 3..4
// replica of the spins), grid.z = gi * 2 + colour.
template <int M>
__global__ __launch_bounds__(256) void msc_init_kernel(MscLattice lat, MscGeom g, uint32_t k0, uint32_t k1,
                                                       uint32_t sample0, uint64_t pcut)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= g.q) return;
    const int what = blockIdx.y;
    const int gi = blockIdx.z >> 1, c = blockIdx.z & 1;
    const int R4 = g.R >> 2;
    const int row = (int)g.by_r4.div((uint32_t)tid);
    const int xh0 = (tid - row * R4) * 4;
    const int z = (int)g.by_l.div((uint32_t)row), y = row - z * g.L;
    const bool bond = what < 3;
    const uint32_t aux = bond ? (uint32_t)what : 0u;
    const uint32_t w2 = bond ? counter_word2(TAG_BOND, (uint32_t)c, 0u)
                             : counter_word2(TAG_INIT, (uint32_t)c, (uint32_t)(what - 3));
    uint32_t out[4] = {0u, 0u, 0u, 0u};
    for (int bit = 0; bit < 32; ++bit) {
        const int m = bit % M, k = bit / M;
        const uint32_t h = (uint32_t)xh0 + (uint32_t)g.R * ((uint32_t)y + (uint32_t)g.L * (uint32_t)(z + k * g.Lz));
        const Words4 u = philox10(aux, h >> 2, w2, sample0 + (uint32_t)(gi * M + m), k0, k1);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t b = bond ? (uint32_t)((uint64_t)u.v[i] < pcut) : (u.v[i] >> 31);
            out[i] |= b << bit;
        }
    }
    uint32_t *dst = bond ? lat.bonds + msc_bond_plane(g, gi, what, c) : lat.spins + msc_spin_plane(g, gi, what - 3, c);
    *reinterpret_cast<uint4 *>(dst + (size_t)row * g.R + xh0) = make_uint4(out[0], out[1], out[2], out[3]);
}

// --------------------------------------------------------------------------
// One checkerboard half-step (Sec. III, eq. 9) of every sample of the batch.
// Replica r updates colour c = r ^ half (the interlaced order).  One thread
// per four consecutive xh of a row of one replica and word set: for each slab
// k it draws one Philox block whose four words are the shared words of its
// four sites, turns them into per-bit threshold masks, and then decides all
// M S bits of each word with the bit-sliced count of unsatisfied bonds.
//
// Block order.  Blocks go to the 8 XCDs in turn (block b to XCD b mod 8), so
// logical block (b mod 8) n/8 + b/8 gives each XCD a contiguous run of tiles
// -- a z-slab, whose neighbour rows then sit in that XCD's L2 -- and logical
// block 2 tile + r puts the two replicas of a tile side by side, so that their
// reads of the shared couplings meet in L2 (xcd_block).  grid.y = word set.

template <int M>
__global__ __launch_bounds__(256) void msc_half_step_kernel(MscLattice lat, MscGeom g, int half,
                                                            const uint32_t *__restrict__ t_base, uint32_t t_off,
                                                            uint32_t k0, uint32_t k1, uint32_t shared,
                                                            uint32_t thr1, uint32_t thr2, uint32_t thr3)
{
    constexpr int S = 32 / M;
    const int lb = xcd_block(debug_block((int)blockIdx.x, (int)gridDim.x, g.order), (int)gridDim.x);
    const int r = lb & 1;
    const int tid = (lb >> 1) * (int)blockDim.x + (int)threadIdx.x;
    if (tid >= g.q) return;
    const int gi = blockIdx.y;
    const int c = r ^ half;
    const int R4 = g.R >> 2;
    const int row = (int)g.by_r4.div((uint32_t)tid);
    const int xh0 = (tid - row * R4) * 4;
    const int z = (int)g.by_l.div((uint32_t)row), y = row - z * g.L;
    const int par = (y + z + c) & 1;  // x = 2 xh + par on this row
    const int R = g.R;
    const bool top = z == g.Lz - 1, bottom = z == 0;
    const uint32_t t = *t_base + t_off;
    // word offsets within a plane: this thread's four words start at 4 tid
    // (= row R + xh0); neighbour rows differ by +-R (y) and +-L R (z), with
    // the periodic wrap of the reduced lattice
    const int LR = g.L * R;
    const uint32_t at = (uint32_t)tid << 2;
    const uint32_t at_yp = at + (uint32_t)(y == g.L - 1 ? R - LR : R);
    const uint32_t at_ym = at + (uint32_t)(y == 0 ? LR - R : -R);
    const uint32_t at_zp = at + (uint32_t)(top ? LR - g.P : LR);
    const uint32_t at_zm = at + (uint32_t)(bottom ? g.P - LR : -LR);
    const uint32_t row0 = at - (uint32_t)xh0;

    // threshold masks: bit b of mj[i] is set iff site i's shared word of
    // b's slab is below thr_j
    uint32_t m1[4] = {0u, 0u, 0u, 0u}, m2[4] = {0u, 0u, 0u, 0u}, m3[4] = {0u, 0u, 0u, 0u};
    const uint32_t w2 = counter_word2(TAG_SHARED, (uint32_t)c, (uint32_t)r);
#pragma unroll
    for (int k = 0; k < S; ++k) {
        // the full site of slab k: z + k Lz, so its half index is at + k P
        const uint32_t h = at + (uint32_t)(k * g.P);
        const Words4 u = philox10(t, h >> 2, w2, shared, k0, k1);
        const uint32_t slab = M == 32 ? 0xffffffffu : (((1u << (M & 31)) - 1u) << (k * M));
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            m1[i] |= u.v[i] < thr1 ? slab : 0u;
            m2[i] |= u.v[i] < thr2 ? slab : 0u;
            m3[i] |= u.v[i] < thr3 ? slab : 0u;
        }
    }

    // 32-bit word offsets from wave-uniform plane bases (planes hold fewer than 2^32 words)
    const uint32_t edge = row0 + (uint32_t)(par ? (xh0 + 4 == R ? 0 : xh0 + 4) : (xh0 == 0 ? R - 1 : xh0 - 1));
    const uint32_t left = row0 + (uint32_t)(xh0 == 0 ? R - 1 : xh0 - 1);
    {
        uint32_t *own = lat.spins + msc_spin_plane(g, gi, r, c);
        const uint32_t *oth = lat.spins + msc_spin_plane(g, gi, r, c ^ 1);
        const uint32_t *bx_own = lat.bonds + msc_bond_plane(g, gi, 0, c);
        const uint32_t *by_own = lat.bonds + msc_bond_plane(g, gi, 1, c);
        const uint32_t *bz_own = lat.bonds + msc_bond_plane(g, gi, 2, c);
        const uint32_t *bx_oth = lat.bonds + msc_bond_plane(g, gi, 0, c ^ 1);
        const uint32_t *by_oth = lat.bonds + msc_bond_plane(g, gi, 1, c ^ 1);
        const uint32_t *bz_oth = lat.bonds + msc_bond_plane(g, gi, 2, c ^ 1);

        const uint4 s4 = load4_at(own, at);
        const uint4 o4 = load4_at(oth, at);
        const uint32_t oe = load_at(oth, edge);
        const uint4 xo4 = load4_at(bx_oth, at);
        const uint32_t xe = load_at(bx_oth, left);
        const uint4 bx4 = load4_at(bx_own, at), by4 = load4_at(by_own, at), bz4 = load4_at(bz_own, at);
        const uint4 yp4 = load4_at(oth, at_yp), ym4 = load4_at(oth, at_ym);
        const uint4 bym4 = load4_at(by_oth, at_ym);
        const uint4 zp4 = load4_at(oth, at_zp), zm4 = load4_at(oth, at_zm);
        const uint4 bzm4 = load4_at(bz_oth, at_zm);

        const uint32_t Sv[4] = {s4.x, s4.y, s4.z, s4.w};
        const uint32_t O[4] = {o4.x, o4.y, o4.z, o4.w};
        const uint32_t Xo[4] = {xo4.x, xo4.y, xo4.z, xo4.w};
        const uint32_t Bx[4] = {bx4.x, bx4.y, bx4.z, bx4.w}, By[4] = {by4.x, by4.y, by4.z, by4.w};
        const uint32_t Bz[4] = {bz4.x, bz4.y, bz4.z, bz4.w};
        const uint32_t Yp[4] = {yp4.x, yp4.y, yp4.z, yp4.w}, Ym[4] = {ym4.x, ym4.y, ym4.z, ym4.w};
        const uint32_t Bym[4] = {bym4.x, bym4.y, bym4.z, bym4.w};
        const uint32_t Zp[4] = {zp4.x, zp4.y, zp4.z, zp4.w}, Zm[4] = {zm4.x, zm4.y, zm4.z, zm4.w};
        const uint32_t Bzm[4] = {bzm4.x, bzm4.y, bzm4.z, bzm4.w};

        uint32_t out[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t s = Sv[i];
            // x neighbours: on even rows (par = 0) +x shares xh and -x is xh - 1;
            // on odd rows +x is xh + 1 and -x shares xh.  The -x coupling is
            // stored at the -x site.
            const uint32_t xp = par ? (i < 3 ? O[i + 1] : oe) : O[i];
            const uint32_t xm = par ? O[i] : (i > 0 ? O[i - 1] : oe);
            const uint32_t bxm = par ? Xo[i] : (i > 0 ? Xo[i - 1] : xe);
            const uint32_t zp = top ? from_slab_above<M>(Zp[i]) : Zp[i];
            const uint32_t zm = bottom ? from_slab_below<M>(Zm[i]) : Zm[i];
            const uint32_t bzm = bottom ? from_slab_below<M>(Bzm[i]) : Bzm[i];
            const Decision d = classify(xor3(s, xp, Bx[i]), xor3(s, xm, bxm), xor3(s, Yp[i], By[i]),
                                        xor3(s, Ym[i], Bym[i]), xor3(s, zp, Bz[i]), xor3(s, zm, bzm));
            // n >= 2 -> thr1 (n >= 3 is in "always"), n = 1 -> thr2, n = 0 -> thr3
            const uint32_t low = __builtin_amdgcn_bitop3_b32(d.odd, m2[i], m3[i], kBitopSelect);
            const uint32_t pick = __builtin_amdgcn_bitop3_b32(d.any, m1[i], low, kBitopSelect);
            out[i] = s ^ (d.always | pick);
        }
        *reinterpret_cast<uint4 *>(own + at) = make_uint4(out[0], out[1], out[2], out[3]);
    }
}

// --------------------------------------------------------------------------
// Measurements (eqs. 1, 2, 3, 7) sample by sample.  Every bit of a word is a
// different (sample, slab), so the sums are per-bit counts.  Each lane visits
// words and adds every per-bit quantity into a bit-sliced counter: eight
// planes holding, bit by bit, the binary digits of a count up to 255.  Every
// 255 words, and at the end, each plane is counted across the wave with one
// ballot per bit, weighted 2^j for plane j, into lane b's accumulator of bit
// b.  The block adds its waves' accumulators in LDS and then to the device
// counters, laid out [quantity][G][32 bits]; the host adds the S bits k M + m
// of each sample m.
enum { MSC_UNSAT = 0, MSC_DOWN = 2, MSC_QDIFF = 4, MSC_AUTO = 5 };

constexpr int kPlanes = 8;
constexpr int kPlaneMax = (1 << kPlanes) - 1;

struct BitCounter {
    uint32_t c[kPlanes];
};

__device__ __forceinline__ void bc_zero(BitCounter &k)
{
#pragma unroll
    for (int j = 0; j < kPlanes; ++j) k.c[j] = 0u;
}

// Ripple-carry add of one bit per position.
__device__ __forceinline__ void bc_add(BitCounter &k, uint32_t x)
{
#pragma unroll
    for (int j = 0; j < kPlanes; ++j) {
        const uint32_t carry = k.c[j] & x;
        k.c[j] ^= x;
        x = carry;
    }
}

// Lane b (< 32) of acc gains the wave's total count of bit b; the counter is cleared.
__device__ __forceinline__ void bc_flush(BitCounter &k, uint32_t &acc)
{
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (int j = 0; j < kPlanes; ++j) {
#pragma unroll
        for (uint32_t b = 0; b < 32; ++b) {
            const uint32_t n = (uint32_t)__popcll(__ballot((k.c[j] >> b) & 1u));
            acc += lane == b ? (n << j) : 0u;
        }
        k.c[j] = 0u;
    }
}

// Block sum of NQ per-bit accumulators, then one atomic per bit and
// quantity: dst[k] receives quantity k's 32 counts.
template <int NQ>
__device__ __forceinline__ void block_flush(const uint32_t (&acc)[NQ], unsigned long long *const (&dst)[NQ])
{
    __shared__ uint32_t red[NQ][32];
    for (int i = threadIdx.x; i < NQ * 32; i += blockDim.x) red[i / 32][i % 32] = 0u;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    if (lane < 32)
#pragma unroll
        for (int k = 0; k < NQ; ++k)
            if (acc[k]) atomicAdd(&red[k][lane], acc[k]);
    __syncthreads();
    for (int i = threadIdx.x; i < NQ * 32; i += blockDim.x)
        if (red[i / 32][i % 32]) atomicAdd(dst[i / 32] + (i % 32), (unsigned long long)red[i / 32][i % 32]);
}

// Walk over the 2P words of a word set (colour-major, then z, y, xh) with a
// fixed stride, the coordinates kept by carries instead of divisions.
struct MscWalk {
    int xh, y, z, c;
    int dxh, dy, dz, dc;

    __device__ __forceinline__ void init(const MscGeom &g, int start, int stride)
    {
        xh = start % g.R;
        int rem = start / g.R;
        y = rem % g.L;
        rem /= g.L;
        z = rem % g.Lz;
        c = rem / g.Lz;
        dxh = stride % g.R;
        rem = stride / g.R;
        dy = rem % g.L;
        rem /= g.L;
        dz = rem % g.Lz;
        dc = rem / g.Lz;
    }
    __device__ __forceinline__ void next(const MscGeom &g)
    {
        xh += dxh;
        int carry = xh >= g.R;
        xh -= carry ? g.R : 0;
        y += dy + carry;
        carry = y >= g.L;
        y -= carry ? g.L : 0;
        z += dz + carry;
        carry = z >= g.Lz;
        z -= carry ? g.Lz : 0;
        c += dc + carry;
    }
    __device__ __forceinline__ bool live() const { return c < 2; }
};

// grid.y = 0: unsatisfied bonds, down spins and the overlap; grid.y = 1 + k:
// the autocorrelation with slot k.  grid.z = word set.
template <int M>
__global__ __launch_bounds__(256) void msc_measure_kernel(MscLattice lat, MscGeom g, const uint32_t *snaps,
                                                          size_t snap_words, int n_sets,
                                                          unsigned long long *acc)
{
    const int gi = blockIdx.z;
    const int what = blockIdx.y;
    const int R = g.R;
    const int stride = gridDim.x * blockDim.x;
    const int n_it = (2 * g.P + stride - 1) / stride;
    MscWalk w;
    w.init(g, blockIdx.x * blockDim.x + threadIdx.x, stride);
    const size_t sstride = (size_t)n_sets * 32;
    unsigned long long *base = acc + (size_t)gi * 32;
    if (what == 0) {
        BitCounter k[5];
        uint32_t cnt[5] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll
        for (int q = 0; q < 5; ++q) bc_zero(k[q]);
        for (int it = 0, run = 0; it < n_it; ++it) {
            // every lane reaches the flushes; lanes past the end add zeros
            uint32_t s0 = 0u, s1 = 0u, un0[3] = {0u, 0u, 0u}, un1[3] = {0u, 0u, 0u};
            if (w.live()) {
                const int c = w.c;
                const int row = w.y + g.L * w.z;
                const size_t hw = (size_t)row * R + w.xh;
                const int par = (w.y + w.z + c) & 1;
                s0 = lat.spins[msc_spin_plane(g, gi, 0, c) + hw];
                s1 = lat.spins[msc_spin_plane(g, gi, 1, c) + hw];
                // bonds to +x, +y, +z, each counted at the site that stores it
                const int xn = par ? (w.xh + 1 == R ? 0 : w.xh + 1) : w.xh;
                const bool top = w.z + 1 == g.Lz;
                const size_t nb[3] = {(size_t)row * R + xn,
                                      (size_t)((w.y + 1 == g.L ? 0 : w.y + 1) + g.L * w.z) * R + w.xh,
                                      (size_t)(w.y + g.L * (top ? 0 : w.z + 1)) * R + w.xh};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const uint32_t J = lat.bonds[msc_bond_plane(g, gi, d, c) + hw];
                    uint32_t n0 = lat.spins[msc_spin_plane(g, gi, 0, c ^ 1) + nb[d]];
                    uint32_t n1 = lat.spins[msc_spin_plane(g, gi, 1, c ^ 1) + nb[d]];
                    if (d == 2 && top) {
                        n0 = from_slab_above<M>(n0);
                        n1 = from_slab_above<M>(n1);
                    }
                    un0[d] = xor3(s0, n0, J);
                    un1[d] = xor3(s1, n1, J);
                }
            }
            w.next(g);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                bc_add(k[0], un0[d]);
                bc_add(k[1], un1[d]);
            }
            bc_add(k[2], s0);
            bc_add(k[3], s1);
            bc_add(k[4], s0 ^ s1);
            // three unsatisfied-bond words per site: flush before 255 can be passed
            if (++run == kPlaneMax / 3 || it + 1 == n_it) {
                run = 0;
#pragma unroll
                for (int q = 0; q < 5; ++q) bc_flush(k[q], cnt[q]);
            }
        }
        unsigned long long *const dst[5] = {base + MSC_UNSAT * sstride, base + (MSC_UNSAT + 1) * sstride,
                                            base + MSC_DOWN * sstride, base + (MSC_DOWN + 1) * sstride,
                                            base + MSC_QDIFF * sstride};
        block_flush<5>(cnt, dst);
    } else {
        const uint32_t *snap = snaps + (size_t)(what - 1) * snap_words;
        BitCounter k[2];
        uint32_t cnt[2] = {0u, 0u};
        bc_zero(k[0]);
        bc_zero(k[1]);
        for (int it = 0, run = 0; it < n_it; ++it) {
            uint32_t d0 = 0u, d1 = 0u;
            if (w.live()) {
                const size_t hw = (size_t)(w.y + g.L * w.z) * R + w.xh;
                const size_t p0 = msc_spin_plane(g, gi, 0, w.c) + hw, p1 = msc_spin_plane(g, gi, 1, w.c) + hw;
                d0 = lat.spins[p0] ^ snap[p0];
                d1 = lat.spins[p1] ^ snap[p1];
            }
            w.next(g);
            bc_add(k[0], d0);
            bc_add(k[1], d1);
            if (++run == kPlaneMax || it + 1 == n_it) {
                run = 0;
                bc_flush(k[0], cnt[0]);
                bc_flush(k[1], cnt[1]);
            }
        }
        const int kk = what - 1;
        unsigned long long *const dst[2] = {base + (MSC_AUTO + 2 * kk) * sstride,
                                            base + (MSC_AUTO + 2 * kk + 1) * sstride};
        block_flush<2>(cnt, dst);
    }
}

// The overlap word q = S_0 ^ S_1 of every site word, [G][colour][P], for the
// C4 passes (one word read per site instead of two).
__global__ __launch_bounds__(256) void msc_q_kernel(MscLattice lat, MscGeom g, int n_sets, uint32_t *q)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t per_set = 2 * (size_t)g.P;
    if (i >= per_set * (size_t)n_sets) return;
    const size_t gi = i / per_set, k = i - gi * per_set;
    const uint32_t *s = lat.spins + gi * 4 * (size_t)g.P;
    q[i] = s[k] ^ s[per_set + k];  // replica 0's two colour planes, then replica 1's
}

// C4 along axis D (eq. 3): sites whose overlap differs from the overlap
// rho e_D away.  grid.y = rho, grid.z = word set; acc points at axis D's
// block, laid out [rho][G][32].
template <int M, int D>
__global__ __launch_bounds__(256) void msc_c4_kernel(const uint32_t *__restrict__ q, MscGeom g, int n_sets,
                                                     unsigned long long *acc)
{
    const int gi = blockIdx.z;
    const int rho = blockIdx.y;
    const int R = g.R;
    const int stride = gridDim.x * blockDim.x;
    const int n_it = (2 * g.P + stride - 1) / stride;
    const uint32_t *qs = q + (size_t)gi * 2 * (size_t)g.P;
    // a z displacement crosses up_base slab faces, plus one more when the
    // reduced z passes Lz
    const int up_base = rho / g.Lz, z_rem = rho - up_base * g.Lz;
    const int flip = rho & 1;  // an odd displacement lands on the other colour
    MscWalk w;
    w.init(g, blockIdx.x * blockDim.x + threadIdx.x, stride);
    BitCounter k;
    bc_zero(k);
    uint32_t cnt[1] = {0u};
    for (int it = 0, run = 0; it < n_it; ++it) {
        uint32_t diff = 0u;
        if (w.live()) {
            const int row = w.y + g.L * w.z;
            const int base2 = (w.c ^ flip) * g.P;
            int w2, up = 0;
            if constexpr (D == 0) {
                int x2 = 2 * w.xh + ((w.y + w.z + w.c) & 1) + rho;
                x2 -= x2 >= g.L ? g.L : 0;
                w2 = base2 + row * R + (x2 >> 1);
            } else if constexpr (D == 1) {
                int y2 = w.y + rho;
                y2 -= y2 >= g.L ? g.L : 0;
                w2 = base2 + (y2 + g.L * w.z) * R + w.xh;
            } else {
                int z2 = w.z + z_rem;
                const int wrap_z = z2 >= g.Lz;
                z2 -= wrap_z ? g.Lz : 0;
                up = up_base + wrap_z;
                w2 = base2 + (w.y + g.L * z2) * R + w.xh;
            }
            const uint32_t q1 = qs[w.c * g.P + row * R + w.xh];
            diff = q1 ^ from_slabs_above<M>(qs[w2], up);
        }
        w.next(g);
        bc_add(k, diff);
        if (++run == kPlaneMax || it + 1 == n_it) {
            run = 0;
            bc_flush(k, cnt[0]);
        }
    }
    unsigned long long *const dst[1] = {acc + ((size_t)rho * n_sets + gi) * 32};
    block_flush<1>(cnt, dst);
}

}  // namespace ea
