// ea_fft.h -- full-vector C4 shells (eq. 3 over every displacement r)
// through the Wiener-Khinchin theorem, for L = 2^k (8 .. 256) and L = 3 2^k
// (24 .. 192): with F the 3D DFT of q = S_0 S_1, the unnormalised inverse DFT
// of |F|^2 is N sum_x q(x) q(x + r) for every r at once.  Five passes over a
// complex fp64 array of L^3 elements, each transforming whole lines of one
// axis in LDS, replace the direct kernel's L^6 / 64 word operations by
// O(L^3 log L) flops and 128 bytes of HBM traffic per site.
//
// The forward transforms are decimation in frequency (natural order in,
// digit-reversed order out along each axis: for L = 3P a radix-3 stage of
// span P first, then radix-2 stages on each third) and the inverse ones
// decimation in time (digit-reversed in, natural out: the same stages in the
// opposite order); |F|^2 is taken pointwise in between, so no pass permutes
// its data.  The autocorrelation is even, so the last two passes transform
// only the planes z <= L/2.  The sums are integers of magnitude <= N and the
// rounding error of the fp64 transforms is ~1e-16 log2(N) of the largest
// |F|^2 (<= N^2), i.e. below 1e-7 after the division by N at L = 256: each
// sum is rounded to the nearest integer, and a sum found farther than 1/4
// from an integer sets an error word instead of being trusted.
#pragma once

#include <hip/hip_runtime.h>

namespace ea {

constexpr int kFftTile = 2048;  // complex elements held by one workgroup, at most
constexpr int kFftThreads = 256;

// The passes, in order: forward along x from the dense q rows, forward along
// y, forward along z + |.|^2 + inverse along z, inverse along y, inverse along
// x + rounding (fft_bin_kernel); then the shell sums (fft_shell_sum_kernel).
enum FftOp { kFftFwdBitsX = 0, kFftFwdY = 1, kFftSquareZ = 2, kFftInvY = 3, kFftInvBinX = 4 };

struct FftArgs {
    double2 *z;                    // [L^3], element (x, y, z) at (z L + y) L + x
    const unsigned long long *qd;  // dense overlap rows (dense_q_kernel): row y + L z, dw words, bit x set iff q = -1
    int dw;
    int n_shells;
    unsigned long long *shells;  // [n_shells] sums, added to (two's complement)
    unsigned int *err;           // set to 1 if a sum is not within 1/4 of an integer
};

constexpr bool fft_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
constexpr int fft_log2(int n) { return n <= 1 ? 0 : 1 + fft_log2(n / 2); }

// Sides the route takes: 2^k for k = 3 .. 8 and 3 2^k for k = 3 .. 6.
constexpr bool fft_side(int L)
{
    return L >= 8 && L <= 256 && (fft_pow2(L) || (L % 3 == 0 && fft_pow2(L / 3) && L / 3 >= 8));
}

// Lines per workgroup tile: the largest power of two B that divides L (so
// that a row holds whole tiles along x), with B <= L and B L <= kFftTile.
constexpr int fft_lines_per_tile(int L)
{
    int b = 1;
    while (L % (2 * b) == 0 && 2 * b <= L && 2 * b * L <= kFftTile) b *= 2;
    return b;
}

template <int L>
struct FftShape {
    static_assert(fft_side(L), "L = 2^k (8 .. 256) or 3 2^k (24 .. 192)");
    static constexpr bool R3 = !fft_pow2(L);    // one radix-3 stage
    static constexpr int P = R3 ? L / 3 : L;    // the power-of-two blocks of the radix-2 stages
    static constexpr int LOG2P = fft_log2(P);
    static constexpr int SC = L / P;            // stride of a P-point twiddle in the L-point table
    static constexpr int NTW = R3 ? L : L / 2;  // twiddle table entries
    static constexpr int B = fft_lines_per_tile(L);
    static constexpr int LP = L + 1;  // LDS stride of a line (padded against bank conflicts)
};

__device__ __forceinline__ double2 cmul(double2 a, double2 w)
{
    return make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}

__device__ __forceinline__ double2 cmulc(double2 a, double2 w)  // a conj(w)
{
    return make_double2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// The P-point block sb of a tile of lines: block r of line b starts at
// b LP + r P.
template <int L>
__device__ __forceinline__ int fft_block_base(int sb)
{
    using S = FftShape<L>;
    return (sb / S::SC) * S::LP + (sb % S::SC) * S::P;
}

// One radix-2 stage of span h = 2^st on every P-point block of the NL lines.
// DIF: (a, b) -> (a + b, (a - b) w); DIT: t = b conj(w), (a, b) -> (a + t,
// a - t); w = exp(-2 pi i pos / 2h), from the table tw[m] = exp(-2 pi i m / L)
// at m = SC pos P / 2h.
template <int L, int NL, bool DIT>
__device__ __forceinline__ void fft_stage2(double2 *s, const double2 *tw, int st, int tid)
{
    using S = FftShape<L>;
    constexpr int H = S::P / 2;
    const int h = 1 << st;
    for (int t = tid; t < NL * S::SC * H; t += kFftThreads) {
        const int sb = t >> (S::LOG2P - 1), kk = t & (H - 1);
        const int pos = kk & (h - 1);
        double2 *p0 = s + fft_block_base<L>(sb) + (((kk >> st) << (st + 1)) | pos), *p1 = p0 + h;
        const double2 w = tw[S::SC * (pos << (S::LOG2P - 1 - st))];
        const double2 x0 = *p0, x1 = *p1;
        if constexpr (DIT) {
            const double2 u = cmulc(x1, w);
            *p0 = cadd(x0, u);
            *p1 = csub(x0, u);
        } else {
            *p0 = cadd(x0, x1);
            *p1 = cmul(csub(x0, x1), w);
        }
    }
}

// Two radix-2 stages, of spans 2h and h (h = 2^sl), in registers on each
// quad {p, p + h, p + 2h, p + 3h}, p = g 4h + pos, pos < h, of a P-point
// block: the span-2h butterflies pair (p, p + 2h) at position pos and
// (p + h, p + 3h) at pos + h, the span-h ones (p, p + h) and (p + 2h, p + 3h),
// both at pos.  DIF takes span 2h first, DIT span h first; the same as the
// two radix-2 stages in turn, with half the LDS traffic and barriers.
template <int L, int NL, bool DIT>
__device__ __forceinline__ void fft_stage4(double2 *s, const double2 *tw, int sl, int tid)
{
    using S = FftShape<L>;
    constexpr int Q = S::P / 4;
    const int h = 1 << sl;
    for (int t = tid; t < NL * S::SC * Q; t += kFftThreads) {
        const int sb = t >> (S::LOG2P - 2), kk = t & (Q - 1);
        const int pos = kk & (h - 1);
        double2 *p = s + fft_block_base<L>(sb) + (((kk >> sl) << (sl + 2)) | pos);
        const double2 wa0 = tw[S::SC * (pos << (S::LOG2P - 2 - sl))];
        const double2 wa1 = tw[S::SC * ((pos + h) << (S::LOG2P - 2 - sl))];
        const double2 wb = tw[S::SC * (pos << (S::LOG2P - 1 - sl))];
        const double2 x0 = p[0], x1 = p[h], x2 = p[2 * h], x3 = p[3 * h];
        if constexpr (DIT) {
            const double2 u1 = cmulc(x1, wb), u3 = cmulc(x3, wb);
            const double2 y0 = cadd(x0, u1), y1 = csub(x0, u1), y2 = cadd(x2, u3), y3 = csub(x2, u3);
            const double2 v2 = cmulc(y2, wa0), v3 = cmulc(y3, wa1);
            p[0] = cadd(y0, v2);
            p[2 * h] = csub(y0, v2);
            p[h] = cadd(y1, v3);
            p[3 * h] = csub(y1, v3);
        } else {
            const double2 y0 = cadd(x0, x2), y2 = cmul(csub(x0, x2), wa0);
            const double2 y1 = cadd(x1, x3), y3 = cmul(csub(x1, x3), wa1);
            p[0] = cadd(y0, y1);
            p[h] = cmul(csub(y0, y1), wb);
            p[2 * h] = cadd(y2, y3);
            p[3 * h] = cmul(csub(y2, y3), wb);
        }
    }
}

// Three radix-2 stages, of spans 4h, 2h and h (h = 2^sl), in registers on
// each octet {p + m h : m = 0 .. 7}, p = g 8h + pos, pos < h, of a P-point
// block: span 4h pairs (m, m + 4) at positions pos + m h, span 2h pairs
// (m, m + 2) of each half at pos + (m & 1) h, span h pairs (m, m + 1) at
// pos.  DIF takes the spans in decreasing order, DIT in increasing order;
// the same as the three radix-2 stages in turn, with a third of their LDS
// round trips and barriers.
template <int L, int NL, bool DIT>
__device__ __forceinline__ void fft_stage8(double2 *s, const double2 *tw, int sl, int tid)
{
    using S = FftShape<L>;
    constexpr int O = S::P / 8;
    const int h = 1 << sl;
    for (int t = tid; t < NL * S::SC * O; t += kFftThreads) {
        const int sb = t >> (S::LOG2P - 3), kk = t & (O - 1);
        const int pos = kk & (h - 1);
        double2 *p = s + fft_block_base<L>(sb) + (((kk >> sl) << (sl + 3)) | pos);
        double2 x[8], wa[4], wb[2];
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = p[m * h];
#pragma unroll
        for (int m = 0; m < 4; ++m) wa[m] = tw[S::SC * ((pos + m * h) << (S::LOG2P - 3 - sl))];
#pragma unroll
        for (int m = 0; m < 2; ++m) wb[m] = tw[S::SC * ((pos + m * h) << (S::LOG2P - 2 - sl))];
        const double2 wc = tw[S::SC * (pos << (S::LOG2P - 1 - sl))];
        if constexpr (DIT) {
#pragma unroll
            for (int m = 0; m < 8; m += 2) {
                const double2 u = cmulc(x[m + 1], wc);
                x[m + 1] = csub(x[m], u);
                x[m] = cadd(x[m], u);
            }
#pragma unroll
            for (int m = 0; m < 8; m += (m & 1) ? 3 : 1) {  // 0, 1, 4, 5
                const double2 u = cmulc(x[m + 2], wb[m & 1]);
                x[m + 2] = csub(x[m], u);
                x[m] = cadd(x[m], u);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double2 u = cmulc(x[m + 4], wa[m]);
                x[m + 4] = csub(x[m], u);
                x[m] = cadd(x[m], u);
            }
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double2 a = x[m], b = x[m + 4];
                x[m] = cadd(a, b);
                x[m + 4] = cmul(csub(a, b), wa[m]);
            }
#pragma unroll
            for (int m = 0; m < 8; m += (m & 1) ? 3 : 1) {  // 0, 1, 4, 5
                const double2 a = x[m], b = x[m + 2];
                x[m] = cadd(a, b);
                x[m + 2] = cmul(csub(a, b), wb[m & 1]);
            }
#pragma unroll
            for (int m = 0; m < 8; m += 2) {
                const double2 a = x[m], b = x[m + 1];
                x[m] = cadd(a, b);
                x[m + 1] = cmul(csub(a, b), wc);
            }
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) p[m * h] = x[m];
    }
}

// The radix-3 stage of span P = L / 3 on each line: (x0, x1, x2) at
// (pos, pos + P, pos + 2P).  With w3 = exp(-2 pi i / 3) and W = exp(-2 pi i
// / L), DIF writes x0 + x1 + x2, (x0 + w3 x1 + w3^2 x2) W^pos and (x0 + w3^2 x1
// + w3 x2) W^2pos; DIT takes z1 = x1 conj(W^pos), z2 = x2 conj(W^2pos) and
// writes x0 + z1 + z2, x0 + conj(w3) z1 + w3 z2 and x0 + w3 z1 + conj(w3) z2.
template <int L, int NL, bool DIT>
__device__ __forceinline__ void fft_stage3(double2 *s, const double2 *tw, int tid)
{
    using S = FftShape<L>;
    constexpr int P = S::P;
    constexpr double kS3 = 0.86602540378443864676;  // sqrt(3) / 2
    for (int t = tid; t < NL * P; t += kFftThreads) {
        const int b = t / P, pos = t - b * P;
        double2 *p = s + b * S::LP + pos;
        const double2 w1 = tw[pos], w2 = tw[2 * pos];
        double2 x0 = p[0], x1 = p[P], x2 = p[2 * P];
        if constexpr (DIT) {
            x1 = cmulc(x1, w1);
            x2 = cmulc(x2, w2);
        }
        const double2 t1 = cadd(x1, x2), t2 = csub(x1, x2);
        const double2 u = make_double2(x0.x - 0.5 * t1.x, x0.y - 0.5 * t1.y);
        // DIF: -i sqrt(3)/2 (x1 - x2); DIT: +i sqrt(3)/2 (x1 - x2)
        const double2 v = DIT ? make_double2(-kS3 * t2.y, kS3 * t2.x) : make_double2(kS3 * t2.y, -kS3 * t2.x);
        p[0] = cadd(x0, t1);
        if constexpr (DIT) {
            p[P] = cadd(u, v);
            p[2 * P] = csub(u, v);
        } else {
            p[P] = cmul(cadd(u, v), w1);
            p[2 * P] = cmul(csub(u, v), w2);
        }
    }
}

// The whole transform of the NL lines; ends with a barrier.  DIF: the
// radix-3 stage (L = 3P), then spans P/2 .. 1 on each P-point block, three
// stages per round, the last one or two in a radix-4 or radix-2 round; DIT:
// the same rounds in the opposite order, then the radix-3 stage.
template <int L, int NL, bool DIT>
__device__ __forceinline__ void fft_lines(double2 *s, const double2 *tw, int tid)
{
    using S = FftShape<L>;
    constexpr int LOG2P = S::LOG2P;
    if constexpr (DIT) {
        // the mirror of the DIF grouping: the radix-2 or radix-4 remainder on
        // the smallest spans first, then radix-8 rounds
        int st = 0;
        if constexpr (LOG2P % 3 == 1) {
            fft_stage2<L, NL, true>(s, tw, 0, tid);
            __syncthreads();
            st = 1;
        } else if constexpr (LOG2P % 3 == 2) {
            fft_stage4<L, NL, true>(s, tw, 0, tid);
            __syncthreads();
            st = 2;
        }
        for (; st + 2 < LOG2P; st += 3) {
            fft_stage8<L, NL, true>(s, tw, st, tid);
            __syncthreads();
        }
        if constexpr (S::R3) {
            fft_stage3<L, NL, true>(s, tw, tid);
            __syncthreads();
        }
    } else {
        if constexpr (S::R3) {
            fft_stage3<L, NL, false>(s, tw, tid);
            __syncthreads();
        }
        int st = LOG2P - 1;
        for (; st >= 2; st -= 3) {
            fft_stage8<L, NL, false>(s, tw, st - 2, tid);
            __syncthreads();
        }
        if (st >= 1) {
            fft_stage4<L, NL, false>(s, tw, st - 1, tid);
            __syncthreads();
            st -= 2;
        }
        if (st == 0) {
            fft_stage2<L, NL, false>(s, tw, 0, tid);
            __syncthreads();
        }
    }
}

// tw[m] = exp(-2 pi i m / L), m < NTW; the caller synchronises.
template <int L>
__device__ __forceinline__ void fft_twiddles(double2 *tw, int tid)
{
    for (int m = tid; m < FftShape<L>::NTW; m += kFftThreads) {
        double sn, cs;
        sincospi(2.0 * (double)m / (double)L, &sn, &cs);
        tw[m] = make_double2(cs, -sn);
    }
}

// Element j of a workgroup's tile: line b, index i along the axis, and its
// position in the L^3 array.  Along x the tile is B consecutive rows (one
// contiguous run); along y (z) it is B consecutive x of one z (y), so that a
// wave reads runs of B consecutive elements.
template <int L, int AXIS>
__device__ __forceinline__ void fft_element(int w, int j, int &b, int &i, size_t &pos)
{
    constexpr int B = FftShape<L>::B, XB = L / B;  // tiles per row
    if constexpr (AXIS == 0) {
        b = j / L;
        i = j - b * L;
        pos = (size_t)w * B * L + (size_t)j;
    } else {
        b = j % B;
        i = j / B;
        const int o = w / XB, x = (w - o * XB) * B + b;
        pos = AXIS == 1 ? ((size_t)o * L + (size_t)i) * L + (size_t)x : ((size_t)i * L + (size_t)o) * L + (size_t)x;
    }
}

// Passes kFftFwdBitsX .. kFftInvY, one tile per workgroup: L^2 / B tiles,
// except kFftInvY, which needs only the planes z <= L/2 ((L/2 + 1) L / B
// tiles; kFftSquareZ stores only those): the autocorrelation is even, A(-r)
// = A(r), so the shells follow from half of it (fft_bin_kernel).
template <int L, int OP>
__global__ __launch_bounds__(kFftThreads) void fft_pass_kernel(FftArgs a)
{
    using S = FftShape<L>;
    constexpr int B = S::B, TILE = B * L;
    constexpr int AXIS = OP == kFftFwdBitsX ? 0 : (OP == kFftSquareZ ? 2 : 1);
    static_assert(OP != kFftInvBinX, "the last pass is fft_bin_kernel");
    __shared__ double2 s[B * S::LP];
    __shared__ double2 tw[S::NTW];
    const int tid = (int)threadIdx.x, w = (int)blockIdx.x;

    fft_twiddles<L>(tw, tid);
    for (int j = tid; j < TILE; j += kFftThreads) {
        int b, i;
        size_t pos;
        fft_element<L, AXIS>(w, j, b, i, pos);
        double2 v;
        if constexpr (OP == kFftFwdBitsX) {
            const size_t row = (size_t)w * B + (size_t)b;
            const unsigned long long word = a.qd[row * (size_t)a.dw + (size_t)(i >> 6)];
            v = make_double2((word >> (i & 63)) & 1ull ? -1.0 : 1.0, 0.0);
        } else {
            v = a.z[pos];
        }
        s[b * S::LP + i] = v;
    }
    __syncthreads();

    if constexpr (OP == kFftFwdBitsX || OP == kFftFwdY) {
        fft_lines<L, B, false>(s, tw, tid);
    } else if constexpr (OP == kFftSquareZ) {
        fft_lines<L, B, false>(s, tw, tid);
        for (int j = tid; j < TILE; j += kFftThreads) {
            double2 *p = s + (j / L) * S::LP + (j % L);
            const double2 v = *p;
            *p = make_double2(v.x * v.x + v.y * v.y, 0.0);
        }
        __syncthreads();
        fft_lines<L, B, true>(s, tw, tid);
    } else {
        fft_lines<L, B, true>(s, tw, tid);
    }

    for (int j = tid; j < TILE; j += kFftThreads) {
        int b, i;
        size_t pos;
        fft_element<L, AXIS>(w, j, b, i, pos);
        if (OP == kFftSquareZ && i > L / 2) continue;
        a.z[pos] = s[b * S::LP + i];
    }
}

constexpr int kFftBinY = 4;  // y values per workgroup of the last pass

// The sums T(i, y, z) of the last pass, one per |x| = i, |y|, |z| <= L/2,
// at [(z (L/2 + 1) + y) (L/2 + 1) + i], in the planes z > L/2 of the complex
// array (no pass reads those after kFftSquareZ; they hold 16 (L/2 - 1) L^2
// bytes, more than the 8 (L/2 + 1)^3 needed).
template <int L>
__device__ __forceinline__ long long *fft_sums(double2 *z)
{
    static_assert((size_t)16 * (L / 2 - 1) * L * L >= (size_t)8 * (L / 2 + 1) * (L / 2 + 1) * (L / 2 + 1),
                  "the sums fit in the planes z > L/2");
    return reinterpret_cast<long long *>(z + (size_t)(L / 2 + 1) * L * L);
}

// The last transform pass, on the planes z = 0 .. L/2: a workgroup takes
// kFftBinY values y <= L/2 of one z and, for each, the rows y and L - y (one
// row if y is 0 or L/2), transforms them along x (DIT), and for every
// |x| = i <= L/2 stores the rounded sums at x = +-i of both rows as T(i, y, z),
// the sum over the minimum images (+-i, +-y, z).  A row (y, z) and the row
// (L - y, L - z) hold A(x, y, z) and A(-x, y, z), so for 0 < z < L/2 the
// sums count twice for the planes L - z that are not transformed.
template <int L>
__global__ __launch_bounds__(kFftThreads) void fft_bin_kernel(FftArgs a)
{
    using S = FftShape<L>;
    constexpr int H = L / 2, LP = S::LP, NL = 2 * kFftBinY;
    constexpr int YB = (H + 1 + kFftBinY - 1) / kFftBinY;  // workgroups per plane
    constexpr double kInvN = 1.0 / ((double)L * L * L);     // exact for power-of-two L
    __shared__ double2 s[NL * LP];
    __shared__ double2 tw[S::NTW];
    const int tid = (int)threadIdx.x, w = (int)blockIdx.x;
    const int z = w / YB, y0 = (w - z * YB) * kFftBinY;

    fft_twiddles<L>(tw, tid);
    // line 2j: row (y0 + j, z); line 2j + 1: row (L - y0 - j, z) if 0 < y0 + j < L/2
    for (int j = tid; j < NL * L; j += kFftThreads) {
        const int line = j / L, x = j - line * L, y = y0 + (line >> 1);
        const bool mirror = (line & 1) != 0;
        double2 v = make_double2(0.0, 0.0);
        if (y <= H && (!mirror || (y != 0 && y != H)))
            v = a.z[((size_t)z * L + (size_t)(mirror ? L - y : y)) * L + (size_t)x];
        s[line * LP + x] = v;
    }
    __syncthreads();
    fft_lines<L, NL, true>(s, tw, tid);

    const long long weight = (z == 0 || z == H) ? 1 : 2;
    long long *T = fft_sums<L>(a.z);
    for (int t = tid; t < kFftBinY * (H + 1); t += kFftThreads) {
        const int j = t / (H + 1), i = t - j * (H + 1), y = y0 + j;
        if (y > H) continue;
        long long sum = 0;
        bool bad = false;
#pragma unroll
        for (int e = 0; e < 4; ++e) {  // bit 0: x -> L - x, bit 1: y -> L - y
            if ((e & 1) && (i == 0 || i == H)) continue;
            if ((e & 2) && (y == 0 || y == H)) continue;
            const double v = s[(2 * j + (e >> 1)) * LP + ((e & 1) ? L - i : i)].x * kInvN;
            const double r = rint(v);
            bad |= !(fabs(v - r) <= 0.25);  // NaN included
            sum += (long long)r;
        }
        if (bad) atomicOr(a.err, 1u);
        T[((size_t)z * (H + 1) + (size_t)y) * (H + 1) + (size_t)i] = sum * weight;
    }
}

// Shell sums from T: one thread per sorted triple p <= q <= r of |x|, |y|,
// |z| values adds T over the triple's distinct orderings (all of which lie in
// the shell p^2 + q^2 + r^2) in one atomic, a sixth as many as one per
// ordering.  One thread per point of the (L/2 + 1)^3 cube; the others return.
template <int L>
__global__ __launch_bounds__(256) void fft_shell_sum_kernel(FftArgs a)
{
    constexpr int H1 = L / 2 + 1;
    const long long *T = fft_sums<L>(a.z);
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= H1 * H1 * H1) return;
    const int p = t % H1, q = (t / H1) % H1, r = t / (H1 * H1);
    if (p > q || q > r) return;
    const int k = p * p + q * q + r * r;
    if (k >= a.n_shells) return;
    auto at = [T](int i, int y, int z) { return T[((size_t)z * H1 + (size_t)y) * H1 + (size_t)i]; };
    long long sum = at(p, q, r);
    if (p == q && q == r) {
    } else if (p == q) {  // (p, p, r): also (p, r, p), (r, p, p)
        sum += at(p, r, p) + at(r, p, p);
    } else if (q == r) {  // (p, q, q): also (q, p, q), (q, q, p)
        sum += at(q, p, q) + at(q, q, p);
    } else {
        sum += at(p, r, q) + at(q, p, r) + at(q, r, p) + at(r, p, q) + at(r, q, p);
    }
    atomicAdd(a.shells + k, (unsigned long long)sum);
}

}  // namespace ea
