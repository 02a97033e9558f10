// ea_kernels.h -- gfx950 kernels of the plain form: initial state, one
// checkerboard half-step per launch, snapshots and the measurement
// reductions.  Layout and random words are described in ea_device.h.
#pragma once

#include "ea_device.h"

namespace ea {

// Geometry of one packed lattice, passed by value to every kernel.
struct Geom {
    int L;       // side length
    int R;       // sites of one colour per row, L / 2
    int RW;      // words per row
    int rows;    // L * L
    int plane;   // words per colour plane, rows * RW
    uint32_t order = 0;  // debug order of the half-step launches' blocks (debug_block)
};

// Device pointers of one run.
struct Lattice {
    uint32_t *spins;  // [replica 2][colour 2][plane]
    uint32_t *bonds;  // [direction 3][colour 2][plane]
};

__device__ __forceinline__ size_t plane_off(const Geom &g, int a, int c)
{
    return ((size_t)a * 2 + (size_t)c) * (size_t)g.plane;
}

// --------------------------------------------------------------------------
// Initial state (Sec. II): couplings with P(J = -1) = p and two replicas of
// uniformly random spins.  One thread per (row, word) of one colour; grid.y
// selects what is drawn: 0..2 the coupling planes of direction d, 3..4 the
// spins of replica 0 / 1; grid.z the colour.
template <int W>
__global__ __launch_bounds__(256) void init_kernel(Lattice lat, Geom g, uint32_t k0, uint32_t k1,
                                                   uint32_t sample, uint64_t pcut)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= g.plane) return;
    const int what = blockIdx.y;
    const int c = blockIdx.z;
    const int row = tid / g.RW;
    const int w = tid - row * g.RW;
    const uint32_t quad0 = (uint32_t)((row * g.R + w * W) >> 2);
    const bool is_bond = what < 3;
    const uint32_t aux = is_bond ? (uint32_t)what : 0u;
    const uint32_t rep = is_bond ? 0u : (uint32_t)(what - 3);
    const uint32_t c2 = counter_word2(is_bond ? TAG_BOND : TAG_INIT, (uint32_t)c, rep);
    uint32_t bits = 0;
#pragma unroll
    for (int j = 0; j < W / 4; ++j) {
        const Words4 u = philox10(aux, quad0 + (uint32_t)j, c2, sample, k0, k1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t bit = is_bond ? (uint32_t)((uint64_t)u.v[q] < pcut) : (u.v[q] >> 31);
            bits |= bit << (4 * j + q);
        }
    }
    uint32_t *dst = is_bond ? lat.bonds + plane_off(g, what, c) : lat.spins + plane_off(g, what - 3, c);
    dst[tid] = bits;
}

// Bit i set iff u[i] < thr, for all W words (two instructions per site).
template <int J, int W>
__device__ __forceinline__ uint32_t below_words(uint32_t accept, const uint32_t (&u)[W], uint32_t thr)
{
    accept = append_below4(accept, u[4 * J + 3], thr, u[4 * J + 2], thr, u[4 * J + 1], thr, u[4 * J], thr);
    if constexpr (J > 0)
        return below_words<J - 1, W>(accept, u, thr);
    else
        return accept;
}

// The same acceptance as accept_words, cheaper where uphill moves of
// dE >= 8 are rare.  If none of the W random words falls below thr2 (and
// thr3 <= thr2), every site with n = 1 or n = 0 is rejected, and a site with
// n = 2 (any & ~always) flips iff its word is below thr1: one compare and
// one append per site instead of a per-site threshold select.  Lanes where
// some word is below thr2 take the general select, so the decisions are the
// same either way.  Used only while a wave meets such a word rarely (thr2 W
// < 2^24, i.e. 64 W thr2 / 2^32 < 1/4 expected per wave), where both
// branches would otherwise run in most waves, and only in launches with
// several waves per SIMD (SCREEN): a wave that runs alone on its SIMD
// is bound by its chain of dependent instructions, which the screen
// lengthens (measured 9% slower for one L = 128 run, 7-12% faster for 5-16
// runs in one launch).  A separate instantiation, so that the unscreened
// kernels keep their own schedule.
template <int W, bool SCREEN>
__device__ __forceinline__ uint32_t accept_screened(const Decision &d, const uint32_t (&u)[W], uint32_t thr1,
                                                    uint32_t thr2, uint32_t thr3)
{
    if constexpr (!SCREEN) return accept_words<W / 4 - 1, W>(0u, d, u, thr1, thr2, thr3);
    const bool rare = (uint64_t)thr2 * (uint64_t)W < (1ull << 24) && thr3 <= thr2;  // uniform
    if (rare) {
        // the n = 2 compares and a three-way minimum tree (depth 4 for
        // W = 32) are independent, so their latencies overlap
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
    return accept_words<W / 4 - 1, W>(0u, d, u, thr1, thr2, thr3);
}

// --------------------------------------------------------------------------
// One checkerboard half-step (Sec. III, eq. 9) of sweep t = *t_base + t_off
// (the base lives on the device so that a captured graph of sweeps can be
// replayed).  grid.y = replica r, which updates colour c = r ^ half; all six
// neighbours of a colour-c site have colour 1 - c, so every thread reads the
// other colour and writes only its own word.  One thread per (row, word).
template <int W, bool SCREEN>
__device__ __forceinline__ void half_step_word(const Lattice &lat, const Geom &g, int half, uint32_t t, int r,
                                               int tid, uint32_t k0, uint32_t k1, uint32_t sample, uint32_t thr1,
                                               uint32_t thr2, uint32_t thr3)
{
    const int c = r ^ half;
    const int row = tid / g.RW;
    const int w = tid - row * g.RW;
    const int y = row % g.L;
    const int z = row / g.L;
    const int par = (y + z + c) & 1;  // x = 2 xh + par on this row
    const int wm = w == 0 ? g.RW - 1 : w - 1;
    const int wp = w == g.RW - 1 ? 0 : w + 1;
    const int row_ym = wrap(y - 1, g.L) + g.L * z, row_yp = wrap(y + 1, g.L) + g.L * z;
    const int row_zm = y + g.L * wrap(z - 1, g.L), row_zp = y + g.L * wrap(z + 1, g.L);

    uint32_t *own = lat.spins + plane_off(g, r, c);
    const uint32_t *oth = lat.spins + plane_off(g, r, c ^ 1);
    const uint32_t *bx_own = lat.bonds + plane_off(g, 0, c);
    const uint32_t *by_own = lat.bonds + plane_off(g, 1, c);
    const uint32_t *bz_own = lat.bonds + plane_off(g, 2, c);
    const uint32_t *bx_oth = lat.bonds + plane_off(g, 0, c ^ 1);
    const uint32_t *by_oth = lat.bonds + plane_off(g, 1, c ^ 1);
    const uint32_t *bz_oth = lat.bonds + plane_off(g, 2, c ^ 1);

    const int base = row * g.RW;
    const uint32_t S = own[base + w];
    const uint32_t O = oth[base + w], Om = oth[base + wm], Op = oth[base + wp];
    const uint32_t Xo = bx_oth[base + w], Xom = bx_oth[base + wm];
    const uint32_t Bx = bx_own[base + w], By = by_own[base + w], Bz = bz_own[base + w];
    const uint32_t Yp = oth[row_yp * g.RW + w], Ym = oth[row_ym * g.RW + w], Bym = by_oth[row_ym * g.RW + w];
    const uint32_t Zp = oth[row_zp * g.RW + w], Zm = oth[row_zm * g.RW + w], Bzm = bz_oth[row_zm * g.RW + w];

    // the random words do not depend on the lattice: computed here, they
    // overlap the latency of the loads above (the scheduling barrier keeps
    // every load issued before them)
    __builtin_amdgcn_sched_barrier(0);
    uint32_t u[W];
    random_words<W / 4 - 1, W>(t, (uint32_t)((row * g.R + w * W) >> 2),
                               counter_word2(TAG_METRO, (uint32_t)c, (uint32_t)r), sample, k0, k1, u);

    // x neighbours: on even rows (par = 0) the +x neighbour shares xh and the
    // -x neighbour sits at xh - 1; on odd rows the +x neighbour is at xh + 1
    // and the -x neighbour shares xh.  The -x bond is stored at the -x site.
    // (selected with a mask rather than a branch, so that no load waits
    // inside a divergent branch before the random words are computed)
    const uint32_t pm = 0u - (uint32_t)par;
    const uint32_t xp = __builtin_amdgcn_bitop3_b32(pm, take_plus1<W>(O, Op), O, kBitopSelect);
    const uint32_t xm = __builtin_amdgcn_bitop3_b32(pm, O ^ Xo, take_minus1<W>(O ^ Xo, Om ^ Xom), kBitopSelect);
    const uint32_t a1 = S ^ xp ^ Bx;
    const uint32_t a2 = S ^ xm;
    const uint32_t a3 = xor3(S, Yp, By);
    const uint32_t a4 = xor3(S, Ym, Bym);
    const uint32_t a5 = xor3(S, Zp, Bz);
    const uint32_t a6 = xor3(S, Zm, Bzm);

    const Decision d = classify(a1, a2, a3, a4, a5, a6);
    // register selects, no LDS table: a table would add a fill and a barrier
    // to every block of a launch this short
    const uint32_t flips = d.always | accept_screened<W, SCREEN>(d, u, thr1, thr2, thr3);
    own[base + w] = S ^ flips;
}

template <int W, bool SCREEN>
__global__ __launch_bounds__(256) void half_step_kernel(Lattice lat, Geom g, int half,
                                                        const uint32_t *__restrict__ t_base, uint32_t t_off,
                                                        uint32_t k0, uint32_t k1, uint32_t sample,
                                                        uint32_t thr1, uint32_t thr2, uint32_t thr3)
{
    const int blk = debug_block((int)blockIdx.x, (int)gridDim.x, g.order);
    const int tid = xcd_block(blk, (int)gridDim.x) * (int)blockDim.x + (int)threadIdx.x;
    if (tid >= g.plane) return;
    half_step_word<W, SCREEN>(lat, g, half, *t_base + t_off, (int)blockIdx.y, tid, k0, k1, sample, thr1, thr2,
                              thr3);
}

// Several runs of the same geometry in one launch: grid.z = member.  Each
// member keeps its own couplings, key, thresholds and sweep counter, so the
// launch is the members' own half-steps side by side.
constexpr int kGroupMax = 16;

struct GroupMember {
    Lattice lat;
    const uint32_t *t_base;
    uint32_t k0, k1, sample, thr1, thr2, thr3;
};

struct GroupArgs {
    GroupMember m[kGroupMax];
};

template <int W, bool SCREEN>
__global__ __launch_bounds__(256) void group_half_step_kernel(GroupArgs a, Geom g, int half, uint32_t t_off)
{
    const int blk = debug_block((int)blockIdx.x, (int)gridDim.x, g.order);
    const int tid = xcd_block(blk, (int)gridDim.x) * (int)blockDim.x + (int)threadIdx.x;
    if (tid >= g.plane) return;
    const GroupMember &M = a.m[blockIdx.z];
    half_step_word<W, SCREEN>(M.lat, g, half, *M.t_base + t_off, (int)blockIdx.y, tid, M.k0, M.k1, M.sample,
                              M.thr1, M.thr2, M.thr3);
}

// --------------------------------------------------------------------------
// Reductions.  Sums are popcounts (number of set bits); the host turns them
// into the +-1 sums of ea_obs.  Each wave reduces with cross-lane shuffles
// and adds its total to a 64-bit counter (integer, so the result does not
// depend on the order of the atomics).

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void wave_add(unsigned long long *dst, uint32_t v)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, (unsigned long long)v);
}

// The same for a whole 256-thread block: one atomic per block instead of
// one per wave, since every wave of a launch adds into the same few counters
// and atomics on one address serialise.  Every thread of the block calls it,
// the same number of times (it synchronises the block).
__device__ __forceinline__ void block_add(unsigned long long *dst, uint32_t v)
{
    __shared__ uint32_t part[256 / 64];
    v = wave_sum(v);
    __syncthreads();  // the previous call has read part
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(dst, (unsigned long long)t);
    }
}

// Counter layout of one measurement (all uint64):
//   [0,1] unsatisfied bonds of replica 0/1
//   [2,3] spins with S = -1, replica 0/1
//   [4]   sites with S_0 != S_1
//   [5 + 2k + r] sites with S_r(t) != S_r(tw_k)
// followed by the C4 block: [c4_base + d (R+1) + rho] sites with q(s) != q(s + rho e_d).
enum { M_UNSAT = 0, M_DOWN = 2, M_QDIFF = 4, M_AUTO = 5 };

// One thread per (colour, row, word) of the whole lattice: grid.x covers
// 2 * plane threads.  snaps = [slot][replica][colour][plane].
template <int W>
__global__ __launch_bounds__(256) void measure_kernel(Lattice lat, Geom g, const uint32_t *snaps,
                                                      int n_slots, unsigned long long *acc)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = gid < 2 * g.plane;
    const int c = live ? gid / g.plane : 0;
    const int tid = live ? gid - c * g.plane : 0;
    const int row = tid / g.RW;
    const int w = tid - row * g.RW;
    const int y = row % g.L;
    const int z = row / g.L;
    const int par = (y + z + c) & 1;
    const int wp = w == g.RW - 1 ? 0 : w + 1;
    const int row_yp = wrap(y + 1, g.L) + g.L * z;
    const int row_zp = y + g.L * wrap(z + 1, g.L);
    const int base = row * g.RW;

    uint32_t S[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const uint32_t *own = lat.spins + plane_off(g, r, c);
        const uint32_t *oth = lat.spins + plane_off(g, r, c ^ 1);
        S[r] = live ? own[base + w] : 0u;
        uint32_t unsat = 0;
        if (live) {
            const uint32_t O = oth[base + w], Op = oth[base + wp];
            const uint32_t xp = par ? take_plus1<W>(O, Op) : O;
            unsat = __popc(S[r] ^ xp ^ lat.bonds[plane_off(g, 0, c) + base + w]) +
                    __popc(xor3(S[r], oth[row_yp * g.RW + w], lat.bonds[plane_off(g, 1, c) + base + w])) +
                    __popc(xor3(S[r], oth[row_zp * g.RW + w], lat.bonds[plane_off(g, 2, c) + base + w]));
        }
        block_add(acc + M_UNSAT + r, unsat);
        block_add(acc + M_DOWN + r, __popc(S[r]));
    }
    block_add(acc + M_QDIFF, __popc(S[0] ^ S[1]));
    for (int k = 0; k < n_slots; ++k) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const uint32_t ref = live ? snaps[((size_t)k * 2 + r) * 2 * g.plane + plane_off(g, 0, c) + tid] : 0u;
            block_add(acc + M_AUTO + 2 * k + r, __popc(S[r] ^ ref));
        }
    }
}

// q = S_0 xor S_1 of word w of a packed row.
__device__ __forceinline__ uint32_t q_word(const Lattice &lat, const Geom &g, int c, int row, int w)
{
    const size_t i = (size_t)row * g.RW + (size_t)w;
    return lat.spins[plane_off(g, 0, c) + i] ^ lat.spins[plane_off(g, 1, c) + i];
}

// C4 block (eq. 3): one thread per (colour, row) and chunk of kC4Rho
// consecutive displacements rho along one axis d; grid.y = d nchunk + chunk,
// nchunk = ceil((R + 1) / kC4Rho).  The thread reads each of its q words once
// and compares it with the partner word of every rho of its chunk, then each
// rho's count is summed over the wave.  The partner of site (x,y,z) is
// (x,y,z) + rho e_d, of colour c ^ (rho & 1).  Along y and z it sits at the
// same half index of the partner row; along x, on a row with x = 2 xh + par,
// its half index is xh + rho/2 (rho even) or xh + (rho-1)/2 + par (rho odd),
// modulo R.
constexpr int kC4Rho = 8;

__host__ __device__ constexpr int c4_chunks(int R) { return (R + kC4Rho) / kC4Rho; }

template <int W>
__global__ __launch_bounds__(256) void c4_kernel(Lattice lat, Geom g, unsigned long long *acc)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = gid < 2 * g.rows;
    const int nchunk = c4_chunks(g.R);
    const int d = blockIdx.y / nchunk;
    const int r0 = (blockIdx.y - d * nchunk) * kC4Rho;
    uint32_t diff[kC4Rho];
#pragma unroll
    for (int k = 0; k < kC4Rho; ++k) diff[k] = 0u;
    if (live) {
        const int c = gid / g.rows;
        const int row = gid - c * g.rows;
        const int y = row % g.L;
        const int z = row / g.L;
        const int par = (y + z + c) & 1;
        for (int w = 0; w < g.RW; ++w) {
            const uint32_t own = q_word(lat, g, c, row, w);
#pragma unroll
            for (int k = 0; k < kC4Rho; ++k) {
                const int rho = r0 + k;
                if (rho > g.R) break;  // uniform: the chunk's tail past R
                const int cp = c ^ (rho & 1);
                if (d == 0) {
                    const int kx = (rho & 1) ? (rho - 1) / 2 + par : rho / 2;
                    const int start = (w * W + kx) % g.R;
                    const int wi = start / W;
                    const int off = start - wi * W;
                    const uint32_t lo = q_word(lat, g, cp, row, wi);
                    const uint32_t hi = q_word(lat, g, cp, row, wi + 1 == g.RW ? 0 : wi + 1);
                    const uint32_t win = off == 0 ? lo : (((lo >> off) | (hi << (W - off))) & word_mask<W>());
                    diff[k] += __popc(own ^ win);
                } else {
                    const int prow = d == 1 ? (y + rho) % g.L + g.L * z : y + g.L * ((z + rho) % g.L);
                    diff[k] += __popc(own ^ q_word(lat, g, cp, prow, w));
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kC4Rho; ++k)
        if (r0 + k <= g.R) block_add(acc + d * (g.R + 1) + r0 + k, diff[k]);
}

// --------------------------------------------------------------------------
// Full-vector C4 (eq. 3 over every displacement r), summed by minimum-image
// distance shells k = |r|^2.  q = S_0 xor S_1 is first rewritten in natural
// x order, one doubled row per (y, z): bits [0, L) hold x = 0..L-1 and bits
// [L, 2L) repeat them, in dw 64-bit words, so that the row shifted
// cyclically by rx is the window of L bits starting at bit rx.

// One thread per (row, word of the doubled row).
template <int W>
__global__ __launch_bounds__(256) void dense_q_kernel(Lattice lat, Geom g, int dw, unsigned long long *qd)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= g.rows * dw) return;
    const int row = gid / dw;
    const int j = gid - row * dw;
    const int y = row % g.L;
    const int z = row / g.L;
    unsigned long long bits = 0;
    for (int b = 0; b < 64; ++b) {
        const int gbit = 64 * j + b;
        if (gbit >= 2 * g.L) break;
        const int x = gbit % g.L;
        const int c = (x + y + z) & 1;
        const int xh = x >> 1;
        const size_t word = (size_t)row * g.RW + (size_t)(xh / W);
        const int bit = xh % W;
        const uint32_t s0 = lat.spins[plane_off(g, 0, c) + word], s1 = lat.spins[plane_off(g, 1, c) + word];
        bits |= (unsigned long long)(((s0 ^ s1) >> bit) & 1u) << b;
    }
    qd[gid] = bits;
}

constexpr int kShellRx = 16;  // displacements along x per workgroup

__device__ __forceinline__ int min_image_sq(int r, int L)
{
    const int m = r < L - r ? r : L - r;
    return m * m;
}

// Workgroup (rx chunk, ry + L rz): every thread takes source rows with a
// stride, holds the source row (NW words) and the partner row at
// (y + ry, z + rz) (doubled, 2 NW words) in registers, counts the sites where
// q differs from q at x + r for the kShellRx displacements rx of the chunk,
// the workgroup adds the counts, and sum_x q(x) q(x + r) = N - 2 * count is
// added to the shell of r.  NW = ceil(L / 64) words per row (L <= 128).
template <int NW>
__global__ __launch_bounds__(256) void c4_shell_kernel(const unsigned long long *qd, int L, int n_shells,
                                                       unsigned long long *shells)
{
    constexpr int DW = 2 * NW;  // words of a doubled row
    __shared__ unsigned int part[kShellRx][256 / 64];
    const int rx0 = blockIdx.x * kShellRx;
    const int ry = (int)(blockIdx.y % (unsigned)L), rz = (int)(blockIdx.y / (unsigned)L);
    const int kyz = min_image_sq(ry, L) + min_image_sq(rz, L);
    int kmin = 1 << 30;
    for (int i = 0; i < kShellRx; ++i)
        if (rx0 + i < L) kmin = min(kmin, kyz + min_image_sq(rx0 + i, L));
    if (kmin >= n_shells) return;  // whole workgroup: no barrier passed yet
    const int tail = L - 64 * (NW - 1);  // bits used in the last word of a row
    const unsigned long long last_mask = tail == 64 ? ~0ull : ((1ull << tail) - 1ull);
    unsigned int cnt[kShellRx];
#pragma unroll
    for (int i = 0; i < kShellRx; ++i) cnt[i] = 0;
    const int rows = L * L;
    for (int row = (int)threadIdx.x; row < rows; row += (int)blockDim.x) {
        const int y = row % L, z = row / L;
        const int prow = (y + ry) % L + L * ((z + rz) % L);
        unsigned long long src[NW], par[DW];
#pragma unroll
        for (int j = 0; j < NW; ++j) src[j] = qd[(size_t)row * DW + j];
#pragma unroll
        for (int j = 0; j < DW; ++j) par[j] = qd[(size_t)prow * DW + j];
#pragma unroll
        for (int i = 0; i < kShellRx; ++i) {
            const int rx = rx0 + i;  // uniform across the workgroup
            if (rx >= L) break;
            const int w0 = rx >> 6, off = rx & 63;
            unsigned int c = 0;
#pragma unroll
            for (int j = 0; j < NW; ++j) {
                // words w0 + j and w0 + j + 1 of the doubled row (w0 is 0 or 1)
                unsigned long long lo = par[j], hi = j + 1 < DW ? par[j + 1] : 0ull;
                if (NW > 1 && w0 == 1) {
                    lo = par[j + 1];
                    hi = j + 2 < DW ? par[j + 2] : 0ull;
                }
                const unsigned long long win = off ? ((lo >> off) | (hi << (64 - off))) : lo;
                unsigned long long d = src[j] ^ win;
                if (j == NW - 1) d &= last_mask;
                c += (unsigned int)__popcll(d);
            }
            cnt[i] += c;
        }
    }
    // workgroup sums: within a wave by shuffles, then across the four waves
#pragma unroll
    for (int i = 0; i < kShellRx; ++i) {
        const uint32_t v = wave_sum(cnt[i]);
        if ((threadIdx.x & 63) == 0) part[i][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < kShellRx) {
        const int i = (int)threadIdx.x;
        const int rx = rx0 + i;
        const int k = kyz + min_image_sq(rx, L);
        if (rx < L && k < n_shells) {
            unsigned long long diff = 0;
            for (int w = 0; w < (int)(blockDim.x / 64); ++w) diff += part[i][w];
            const long long n = (long long)L * L * L;
            atomicAdd(shells + k, (unsigned long long)(n - 2 * (long long)diff));
        }
    }
}

// Plain word copy (snapshots) and fill (clearing counters); kernels rather
// than runtime memset/memcpy so that the same work can sit in a graph.
__global__ __launch_bounds__(256) void copy_words_kernel(uint32_t *dst, const uint32_t *src, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void zero_u64_kernel(unsigned long long *dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = 0ull;
}

__global__ __launch_bounds__(256) void zero_u32_kernel(uint32_t *dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = 0u;
}

// Device-side sweep counter: set it, or advance it after a block of sweeps.
__global__ void set_u32_kernel(uint32_t *dst, uint32_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v;
}

__global__ void advance_u32_kernel(uint32_t *dst, uint32_t k)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst += k;
}

}  // namespace ea
