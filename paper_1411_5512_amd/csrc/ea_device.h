// ea_device.h -- device-side building blocks shared by the gfx950 kernels:
// the counter-based random words, the packed lattice layout and the
// bit-sliced Metropolis decision.
//
// Packed layout.  Each colour c of each replica is stored as L*L rows, one
// per (y, z), row index y + L z.  A row holds the R = L/2 sites of colour c
// with that (y, z), ordered by xh = x >> 1 (so x = 2 xh + ((y + z + c) & 1)),
// split into RW words of W bits (R = W RW, W a multiple of 4, at most 32);
// bit b of word w is the site xh = W w + b, and bits W..31 are zero.  Spins
// carry 1 for S = -1, couplings 1 for J = -1; a site's three couplings to its
// +x, +y, +z neighbours ("left/up" bonds, Sec. III) live in three planes
// laid out like the spins of the site's colour.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ea {

// ---------------------------------------------------------------------------
// Counter-based random words: Philox4x32-10 (Salmon et al., SC'11).  The key
// is the run's seed, the counter names what the words are for; see ea.h for
// the keying.  Key and the upper counter words are wave-uniform, so the
// compiler keeps them (and the first round's product of word 2) in SGPRs.

struct Words4 {
    uint32_t v[4];
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words4 philox10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                           uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t m0 = (uint64_t)x0 * 0xD2511F53u;
        const uint64_t m2 = (uint64_t)x2 * 0xCD9E8D57u;
        const uint32_t y0 = xor3((uint32_t)(m2 >> 32), x1, k0);
        const uint32_t y2 = xor3((uint32_t)(m0 >> 32), x3, k1);
        x1 = (uint32_t)m2;
        x3 = (uint32_t)m0;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Words4 r;
    r.v[0] = x0;
    r.v[1] = x1;
    r.v[2] = x2;
    r.v[3] = x3;
    return r;
}

// Counter word 1 of block J of a packed word of W sites is quad0 + J, where
// quad0 (the word's first 4-site block) is a multiple of W/4: rows and words
// hold whole numbers of blocks.  For W/4 a power of two the sum has no carry
// and equals quad0 | J, which the first round folds into its XOR.
template <int W>
constexpr bool kQuadOr = ((W / 4) & (W / 4 - 1)) == 0;

constexpr int kBitopOrXor = 0x56;  // (src0 | src1) ^ src2, bitwise

// Two blocks whose counters differ only in word 1 (quad0 + Ja, quad0 + Jb),
// computed round by round side by side: the two dependency chains
// interleave, so each round's multiplies of one block issue while the
// other's are in flight.  In the first round words 0, 2, 3 and the key are
// uniform across the wavefront, so only the word-1 XOR is per lane.
template <bool ORQ>
__device__ __forceinline__ void philox10_pair(uint32_t x0, uint32_t quad0, uint32_t Ja, uint32_t Jb, uint32_t x2,
                                              uint32_t x3, uint32_t k0, uint32_t k1, Words4 &a, Words4 &b)
{
    const uint64_t n0 = (uint64_t)x0 * 0xD2511F53u;
    const uint64_t n2 = (uint64_t)x2 * 0xCD9E8D57u;
    const uint32_t h = (uint32_t)(n2 >> 32) ^ k0;
    uint32_t a0, b0;
    if constexpr (ORQ) {
        a0 = __builtin_amdgcn_bitop3_b32(quad0, Ja, h, kBitopOrXor);
        b0 = __builtin_amdgcn_bitop3_b32(quad0, Jb, h, kBitopOrXor);
    } else {
        a0 = (quad0 + Ja) ^ h;
        b0 = (quad0 + Jb) ^ h;
    }
    uint32_t a1 = (uint32_t)n2, a2 = xor3((uint32_t)(n0 >> 32), x3, k1), a3 = (uint32_t)n0;
    uint32_t b1 = a1, b2 = a2, b3 = a3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
#pragma unroll
    for (int round = 1; round < 10; ++round) {
        const uint64_t ma0 = (uint64_t)a0 * 0xD2511F53u, mb0 = (uint64_t)b0 * 0xD2511F53u;
        const uint64_t ma2 = (uint64_t)a2 * 0xCD9E8D57u, mb2 = (uint64_t)b2 * 0xCD9E8D57u;
        const uint32_t ya0 = xor3((uint32_t)(ma2 >> 32), a1, k0), yb0 = xor3((uint32_t)(mb2 >> 32), b1, k0);
        const uint32_t ya2 = xor3((uint32_t)(ma0 >> 32), a3, k1), yb2 = xor3((uint32_t)(mb0 >> 32), b3, k1);
        a1 = (uint32_t)ma2;
        b1 = (uint32_t)mb2;
        a3 = (uint32_t)ma0;
        b3 = (uint32_t)mb0;
        a0 = ya0;
        b0 = yb0;
        a2 = ya2;
        b2 = yb2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    a.v[0] = a0;
    a.v[1] = a1;
    a.v[2] = a2;
    a.v[3] = a3;
    b.v[0] = b0;
    b.v[1] = b1;
    b.v[2] = b2;
    b.v[3] = b3;
}

enum : uint32_t { TAG_METRO = 0u, TAG_BOND = 1u, TAG_INIT = 2u };

__device__ __forceinline__ uint32_t counter_word2(uint32_t tag, uint32_t colour, uint32_t replica)
{
    return (tag << 8) | (colour << 1) | replica;
}

// ---------------------------------------------------------------------------
// Packed-row helpers.

template <int W>
__device__ __forceinline__ constexpr uint32_t word_mask()
{
    return W >= 32 ? 0xffffffffu : ((1u << W) - 1u);
}

// Word w of a row shifted so that bit b holds site xh - 1 (periodic in R):
// cur = word w, prev = word w-1 (mod RW).
template <int W>
__device__ __forceinline__ uint32_t take_minus1(uint32_t cur, uint32_t prev)
{
    return ((cur << 1) | (prev >> (W - 1))) & word_mask<W>();
}

// Word w of a row shifted so that bit b holds site xh + 1: next = word w+1.
template <int W>
__device__ __forceinline__ uint32_t take_plus1(uint32_t cur, uint32_t next)
{
    return (cur >> 1) | ((next & 1u) << (W - 1));
}

// Workgroups are handed to the 8 XCDs in turn (block b to XCD b mod 8), each
// XCD with its own L2.  Renumbering block b as (b mod 8) n/8 + b/8 gives each
// XCD a contiguous run of logical blocks, so that neighbouring rows of the
// lattice are read through the same L2 (n a multiple of 8; else unchanged).
__device__ __forceinline__ int xcd_block(int b, int n)
{
    return (n & 7) ? b : (b & 7) * (n >> 3) + (b >> 3);
}

// Debug order of a launch's workgroups (ea_set_debug).  order = 0 keeps
// block b; otherwise bit 31 reverses the order and bits 0..30 rotate it.
// Always a permutation of [0, n), so every tile is still taken exactly once.
__device__ __forceinline__ int debug_block(int b, int n, uint32_t order)
{
    if (order == 0) return b;
    if (order & 0x80000000u) b = n - 1 - b;
    return (int)(((uint32_t)b + (order & 0x7fffffffu) % (uint32_t)n) % (uint32_t)n);
}

// Debug fill of LDS words [0, n) (ea_set_debug's poison; 0 = off), so that a
// word read before the kernel wrote it shows up as a wrong result instead of
// a stale value that happens to be right.  The caller synchronises after it.
__device__ __forceinline__ void debug_poison(uint32_t *lds, int n, uint32_t poison, int tid, int nthreads)
{
    if (poison == 0) return;
    for (int i = tid; i < n; i += nthreads) lds[i] = poison ^ (uint32_t)i * 0x01000193u;
}

__device__ __forceinline__ int wrap(int v, int L)
{
    return v < 0 ? v + L : (v >= L ? v - L : v);
}

// ---------------------------------------------------------------------------
// Bit-sliced Metropolis decision for W sites of one colour (eq. 9).
//
// a1..a6 hold, per site, whether each of its six bonds is unsatisfied
// (J S_i S_j = -1).  With n unsatisfied bonds the flip costs dE = 12 - 4n:
// n >= 3 always flips, n = 2, 1, 0 flip iff the site's word is below
// thr1, thr2, thr3.  The counter is reduced with two full adders:
// n = s + 2 (c0 + c1 + c2), so "any" = (c0|c1|c2) means n >= 2 and
// "always" = maj(c0,c1,c2) | (any & s) means n >= 3.
struct Decision {
    uint32_t always;  // n >= 3
    uint32_t any;     // n >= 2
    uint32_t odd;     // n odd
};

__device__ __forceinline__ Decision classify(uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4,
                                             uint32_t a5, uint32_t a6)
{
    const uint32_t s1 = xor3(a1, a2, a3);
    const uint32_t c1 = (a1 & a2) | (a3 & (a1 | a2));
    const uint32_t s2 = xor3(a4, a5, a6);
    const uint32_t c2 = (a4 & a5) | (a6 & (a4 | a5));
    const uint32_t s = s1 ^ s2;
    const uint32_t c0 = s1 & s2;
    const uint32_t any = c0 | c1 | c2;
    const uint32_t two = (c0 & c1) | (c2 & (c0 | c1));
    Decision d;
    d.any = any;
    d.odd = s;
    d.always = two | (any & s);
    return d;
}

// Per-site acceptance, branch-free.  For site bit I the threshold is picked
// with two sign-extended bit fields: any -> thr1 (n = 2), else odd -> thr2
// (n = 1), else thr3 (n = 0); sites with n >= 3 are covered by the "always"
// mask.  The accept word is built from the highest site bit down, one
// Philox block (four sites) at a time, by append_below4.
//
// v_bitop3_b32 truth tables are indexed by (src0 << 2) | (src1 << 1) | src2.
constexpr int kBitopSelect = 0xCA;   // src0 ? src1 : src2, bitwise

// accept = 16 accept + 8 [u3 < t3] + 4 [u2 < t2] + 2 [u1 < t1] + [u0 < t0].
// Each unsigned compare writes its lane mask to an SGPR pair and an add with
// carry-in (accept + accept + carry) appends the bit: two instructions per
// site.  gfx950 needs two wait states between a VALU write of an SGPR and a
// VALU read of it as a carry, so the four compares are issued first: every
// mask is read three instructions after it is written.
__device__ __forceinline__ uint32_t append_below4(uint32_t accept, uint32_t u3, uint32_t t3, uint32_t u2,
                                                  uint32_t t2, uint32_t u1, uint32_t t1, uint32_t u0,
                                                  uint32_t t0)
{
    uint64_t m3, m2, m1, m0, co;
    asm("v_cmp_lt_u32_e64 %1, %6, %7\n\t"
        "v_cmp_lt_u32_e64 %2, %8, %9\n\t"
        "v_cmp_lt_u32_e64 %3, %10, %11\n\t"
        "v_cmp_lt_u32_e64 %4, %12, %13\n\t"
        "v_addc_co_u32_e64 %0, %5, %0, %0, %1\n\t"
        "v_addc_co_u32_e64 %0, %5, %0, %0, %2\n\t"
        "v_addc_co_u32_e64 %0, %5, %0, %0, %3\n\t"
        "v_addc_co_u32_e64 %0, %5, %0, %0, %4"
        : "+v"(accept), "=&s"(m3), "=&s"(m2), "=&s"(m1), "=&s"(m0), "=&s"(co)
        : "v"(u3), "v"(t3), "v"(u2), "v"(t2), "v"(u1), "v"(t1), "v"(u0), "v"(t0));
    return accept;
}

template <int I>
__device__ __forceinline__ uint32_t bit_as_mask(uint32_t word)
{
    // Written as an instruction so that the compiler does not rebuild it as
    // a compare and a lane-mask select.
    uint32_t m;
    asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(m) : "v"(word), "i"(I));
    return m;
}

template <int I>
__device__ __forceinline__ uint32_t site_threshold(const Decision &d, uint32_t thr1, uint32_t thr2, uint32_t thr3)
{
    const uint32_t m_any = bit_as_mask<I>(d.any);
    const uint32_t m_odd = bit_as_mask<I>(d.odd);
    return __builtin_amdgcn_bitop3_b32(m_any, thr1, __builtin_amdgcn_bitop3_b32(m_odd, thr2, thr3, kBitopSelect),
                                       kBitopSelect);
}

// Blocks J = W/4-1 down to 0: block J covers sites 4J..4J+3 and has counter
// word 1 equal to quad0 + J; words 0, 2, 3 (sweep, tag/colour/replica,
// sample) are wave-uniform, so the first rounds run largely on the SALU.
template <int W, int J>
__device__ __forceinline__ uint32_t accept_blocks(uint32_t accept, const Decision &d, uint32_t c0,
                                                  uint32_t quad0, uint32_t c2, uint32_t c3, uint32_t k0,
                                                  uint32_t k1, uint32_t thr1, uint32_t thr2, uint32_t thr3)
{
    if constexpr (J > 0) {
        // blocks J and J - 1 side by side
        Words4 u, v;
        philox10_pair<kQuadOr<W>>(c0, quad0, (uint32_t)J, (uint32_t)(J - 1), c2, c3, k0, k1, u, v);
        accept = append_below4(accept, u.v[3], site_threshold<4 * J + 3>(d, thr1, thr2, thr3), u.v[2],
                               site_threshold<4 * J + 2>(d, thr1, thr2, thr3), u.v[1],
                               site_threshold<4 * J + 1>(d, thr1, thr2, thr3), u.v[0],
                               site_threshold<4 * J + 0>(d, thr1, thr2, thr3));
        accept = append_below4(accept, v.v[3], site_threshold<4 * J - 1>(d, thr1, thr2, thr3), v.v[2],
                               site_threshold<4 * J - 2>(d, thr1, thr2, thr3), v.v[1],
                               site_threshold<4 * J - 3>(d, thr1, thr2, thr3), v.v[0],
                               site_threshold<4 * J - 4>(d, thr1, thr2, thr3));
        if constexpr (J > 1)
            return accept_blocks<W, J - 2>(accept, d, c0, quad0, c2, c3, k0, k1, thr1, thr2, thr3);
        else
            return accept;
    } else {
        const Words4 u = philox10(c0, quad0, c2, c3, k0, k1);
        return append_below4(accept, u.v[3], site_threshold<3>(d, thr1, thr2, thr3), u.v[2],
                             site_threshold<2>(d, thr1, thr2, thr3), u.v[1], site_threshold<1>(d, thr1, thr2, thr3),
                             u.v[0], site_threshold<0>(d, thr1, thr2, thr3));
    }
}

// Flip mask of one packed word of W sites (bits W..31 stay zero).
template <int W>
__device__ __forceinline__ uint32_t flip_mask(const Decision &d, uint32_t c0, uint32_t quad0,
                                              uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                              uint32_t thr1, uint32_t thr2, uint32_t thr3)
{
    return d.always | accept_blocks<W, W / 4 - 1>(0u, d, c0, quad0, c2, c3, k0, k1, thr1, thr2, thr3);
}

// The same flip mask in two steps, for kernels that wait on global loads:
// first the W random words (they depend only on the counter, so they can be
// computed while the neighbour words are in flight), then the decisions.
template <int J, int W>
__device__ __forceinline__ void random_words(uint32_t c0, uint32_t quad0, uint32_t c2, uint32_t c3, uint32_t k0,
                                             uint32_t k1, uint32_t (&u)[W])
{
    if constexpr (J > 0) {
        Words4 a, b;
        philox10_pair<kQuadOr<W>>(c0, quad0, (uint32_t)J, (uint32_t)(J - 1), c2, c3, k0, k1, a, b);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            u[4 * J + i] = a.v[i];
            u[4 * J - 4 + i] = b.v[i];
        }
        if constexpr (J > 1) random_words<J - 2, W>(c0, quad0, c2, c3, k0, k1, u);
    } else {
        const Words4 a = philox10(c0, quad0, c2, c3, k0, k1);
#pragma unroll
        for (int i = 0; i < 4; ++i) u[i] = a.v[i];
    }
}

template <int J, int W>
__device__ __forceinline__ uint32_t accept_words(uint32_t accept, const Decision &d, const uint32_t (&u)[W],
                                                 uint32_t thr1, uint32_t thr2, uint32_t thr3)
{
    accept = append_below4(accept, u[4 * J + 3], site_threshold<4 * J + 3>(d, thr1, thr2, thr3), u[4 * J + 2],
                           site_threshold<4 * J + 2>(d, thr1, thr2, thr3), u[4 * J + 1],
                           site_threshold<4 * J + 1>(d, thr1, thr2, thr3), u[4 * J],
                           site_threshold<4 * J>(d, thr1, thr2, thr3));
    if constexpr (J > 0)
        return accept_words<J - 1, W>(accept, d, u, thr1, thr2, thr3);
    else
        return accept;
}

// ---------------------------------------------------------------------------
// Threshold select through an LDS table, four sites per read.  A 4-site
// block has class bits any (n >= 2) and odd (n odd) for its four sites; the
// byte any_nibble | odd_nibble << 4 indexes a 256-entry table of 16-byte
// entries holding the block's four thresholds (any -> thr1, else odd ->
// thr2, else thr3; a site with n >= 3 is covered by the "always" mask, its
// entry is 0).  The index bytes of all blocks of a word come from two
// interleaves of the class masks: lo = (any & 0x0F0F0F0F) | (odd << 4 &
// 0xF0F0F0F0) holds those of blocks 0, 2, 4, 6, hi = (any >> 4 & 0x0F0F0F0F)
// | (odd & 0xF0F0F0F0) those of blocks 1, 3, 5, 7, so an entry's byte offset
// is one byte extract and shift: per 8 sites one interleave op, two extracts
// and two 16-byte reads.
//
// Layout (words): entry e at [4e, 4e + 4).

constexpr int kSelectTableWords = 4 * 256;

// Fill the table (any thread count; caller synchronises before use).
__device__ __forceinline__ void fill_select_tables(uint32_t *tab, uint32_t thr1, uint32_t thr2, uint32_t thr3,
                                                   int tid, int nthreads)
{
    for (int i = tid; i < kSelectTableWords; i += nthreads) {
        const int idx = i >> 2, q = i & 3;
        const int any = (idx >> q) & 1, odd = (idx >> (4 + q)) & 1;
        tab[i] = any ? (odd ? 0u : thr1) : (odd ? thr2 : thr3);
    }
}

// The W thresholds of one word from the table (16-byte aligned).
template <int W>
__device__ __forceinline__ void select_thresholds(const Decision &d, const uint32_t *tab, uint32_t (&thr)[W])
{
    const uint32_t nib = 0x0F0F0F0Fu;
    const uint32_t lo = __builtin_amdgcn_bitop3_b32(nib, d.any, d.odd << 4, kBitopSelect);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32(nib, d.any >> 4, d.odd, kBitopSelect);
#pragma unroll
    for (int g = 0; g < W / 4; ++g) {
        const uint32_t src = (g & 1) ? hi : lo;
        const uint32_t byte_off = ((src >> (8 * (g >> 1))) & 0xffu) << 4;
        const uint4 q = *(const uint4 *)((const char *)tab + byte_off);
        thr[4 * g + 0] = q.x;
        thr[4 * g + 1] = q.y;
        thr[4 * g + 2] = q.z;
        thr[4 * g + 3] = q.w;
    }
}

template <int J, int W>
__device__ __forceinline__ uint32_t accept_blocks_lds(uint32_t accept, const uint32_t (&thr)[W], uint32_t c0,
                                                      uint32_t quad0, uint32_t c2, uint32_t c3, uint32_t k0,
                                                      uint32_t k1)
{
    if constexpr (J > 0) {
        // blocks J and J - 1 side by side
        Words4 u, v;
        philox10_pair<kQuadOr<W>>(c0, quad0, (uint32_t)J, (uint32_t)(J - 1), c2, c3, k0, k1, u, v);
        accept = append_below4(accept, u.v[3], thr[4 * J + 3], u.v[2], thr[4 * J + 2], u.v[1], thr[4 * J + 1],
                               u.v[0], thr[4 * J]);
        accept = append_below4(accept, v.v[3], thr[4 * J - 1], v.v[2], thr[4 * J - 2], v.v[1], thr[4 * J - 3],
                               v.v[0], thr[4 * J - 4]);
        if constexpr (J > 1)
            return accept_blocks_lds<J - 2, W>(accept, thr, c0, quad0, c2, c3, k0, k1);
        else
            return accept;
    } else {
        const Words4 u = philox10(c0, quad0, c2, c3, k0, k1);
        return append_below4(accept, u.v[3], thr[3], u.v[2], thr[2], u.v[1], thr[1], u.v[0], thr[0]);
    }
}

// Flip mask of one packed word of W sites, thresholds from the LDS table
// (tab = kSelectTableWords words filled by fill_select_tables, 16-byte
// aligned).  All W thresholds are read before the random words are
// computed, so the LDS latency overlaps the Philox rounds.
template <int W>
__device__ __forceinline__ uint32_t flip_mask_lds(const Decision &d, uint32_t c0, uint32_t quad0, uint32_t c2,
                                                  uint32_t c3, uint32_t k0, uint32_t k1, const uint32_t *tab)
{
    uint32_t thr[W];
    select_thresholds<W>(d, tab, thr);
    return d.always | accept_blocks_lds<W / 4 - 1, W>(0u, thr, c0, quad0, c2, c3, k0, k1);
}

}  // namespace ea
