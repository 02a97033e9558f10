// ea_fft.h -- full-vector C4 shells (eq. 3 over every displacement r) for
// power-of-two L through the Wiener-Khinchin theorem: with F the 3D DFT of
// q = S_0 S_1, the unnormalised inverse DFT of |F|^2 is N sum_x q(x) q(x + r)
// for every r at once.  Five passes over a complex fp64 array of L^3
// elements, each transforming whole lines of one axis in LDS with radix-2
// butterflies, replace the direct kernel's L^6 / 64 word operations by
// O(L^3 log L) flops and 128 bytes of HBM traffic per site.
//
// The forward transforms are decimation in frequency (natural order in,
// bit-reversed order out along each axis) and the inverse ones decimation in
// time (bit-reversed in, natural out); |F|^2 is taken pointwise in between,
// so no pass permutes its data.  The autocorrelation is even, so the last two
// passes transform only the planes z <= L/2.  The sums are integers of magnitude <= N and
// the rounding error of the fp64 transforms is ~1e-16 log2(N) of the largest
// |F|^2 (<= N^2), i.e. below 1e-7 after the division by N at L = 256: each
// sum is rounded to the nearest integer, and a sum found farther than 1/4
// from an integer sets an error word instead of being trusted.
#pragma once

#include <hip/hip_runtime.h>

namespace ea {

constexpr int kFftTile = 2048;  // complex elements held by one workgroup
constexpr int kFftThreads = 256;

// The passes, in order: forward along x from the dense q rows, forward along
// y, forward along z + |.|^2 + inverse along z, inverse along y, inverse along
// x + rounding and shell sums (fft_bin_kernel).
enum FftOp { kFftFwdBitsX = 0, kFftFwdY = 1, kFftSquareZ = 2, kFftInvY = 3, kFftInvBinX = 4 };

struct FftArgs {
    double2 *z;                    // [L^3], element (x, y, z) at (z L + y) L + x
    const unsigned long long *qd;  // dense overlap rows (dense_q_kernel): row y + L z, dw words, bit x set iff q = -1
    int dw;
    int n_shells;
    unsigned long long *shells;  // [n_shells] sums, added to (two's complement)
    unsigned int *err;           // set to 1 if a sum is not within 1/4 of an integer
};

template <int LOG2L>
struct FftShape {
    static constexpr int L = 1 << LOG2L;
    static constexpr int B = L < kFftTile / L ? L : kFftTile / L;  // lines per workgroup
    static constexpr int LOG2B = LOG2L < 11 - LOG2L ? LOG2L : 11 - LOG2L;
    static constexpr int LP = L + 1;  // LDS stride of a line (padded against bank conflicts)
    static_assert((1 << LOG2B) == B, "B is a power of two");
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

// One radix-2 stage of span h = 2^st on the NL lines of a tile (stride LP).
// DIF: (a, b) -> (a + b, (a - b) w); DIT: t = b conj(w), (a, b) -> (a + t,
// a - t); w = exp(-2 pi i pos / 2h) = tw[pos L / 2h] from the table tw[m] =
// exp(-2 pi i m / L).
template <int LOG2L, int NL, bool DIT>
__device__ __forceinline__ void fft_stage2(double2 *s, const double2 *tw, int st, int tid)
{
    constexpr int L = 1 << LOG2L, H = L / 2, LP = L + 1;
    const int h = 1 << st;
    for (int t = tid; t < NL * H; t += kFftThreads) {
        const int b = t >> (LOG2L - 1), kk = t & (H - 1);
        const int pos = kk & (h - 1);
        double2 *p0 = s + b * LP + (((kk >> st) << (st + 1)) | pos), *p1 = p0 + h;
        const double2 w = tw[pos << (LOG2L - 1 - st)];
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
// quad {p, p + h, p + 2h, p + 3h}, p = g 4h + pos, pos < h: the span-2h
// butterflies pair (p, p + 2h) at position pos and (p + h, p + 3h) at pos + h,
// the span-h ones (p, p + h) and (p + 2h, p + 3h), both at pos.  DIF takes
// span 2h first, DIT span h first; the same as the two radix-2 stages in
// turn, with half the LDS traffic and barriers.
template <int LOG2L, int NL, bool DIT>
__device__ __forceinline__ void fft_stage4(double2 *s, const double2 *tw, int sl, int tid)
{
    constexpr int L = 1 << LOG2L, Q = L / 4, LP = L + 1;
    const int h = 1 << sl;
    for (int t = tid; t < NL * Q; t += kFftThreads) {
        const int b = t >> (LOG2L - 2), kk = t & (Q - 1);
        const int pos = kk & (h - 1);
        double2 *p = s + b * LP + (((kk >> sl) << (sl + 2)) | pos);
        const double2 wa0 = tw[pos << (LOG2L - 2 - sl)], wa1 = tw[(pos + h) << (LOG2L - 2 - sl)];
        const double2 wb = tw[pos << (LOG2L - 1 - sl)];
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

// The whole transform of the NL lines: DIF spans L/2 .. 1 (natural order in,
// bit-reversed out), DIT spans 1 .. L/2 (bit-reversed in, natural out), two
// stages per round and a radix-2 stage for odd log2 L; ends with a barrier.
template <int LOG2L, int NL, bool DIT>
__device__ __forceinline__ void fft_lines(double2 *s, const double2 *tw, int tid)
{
    if constexpr (DIT) {
        int st = 0;
        for (; st + 1 < LOG2L; st += 2) {
            fft_stage4<LOG2L, NL, true>(s, tw, st, tid);
            __syncthreads();
        }
        if (st < LOG2L) {
            fft_stage2<LOG2L, NL, true>(s, tw, st, tid);
            __syncthreads();
        }
    } else {
        int st = LOG2L - 1;
        for (; st >= 1; st -= 2) {
            fft_stage4<LOG2L, NL, false>(s, tw, st - 1, tid);
            __syncthreads();
        }
        if (st == 0) {
            fft_stage2<LOG2L, NL, false>(s, tw, 0, tid);
            __syncthreads();
        }
    }
}

template <int LOG2L>
__device__ __forceinline__ void fft_twiddles(double2 *tw, int tid)
{
    constexpr int L = 1 << LOG2L;
    for (int m = tid; m < L / 2; m += kFftThreads) {
        double sn, cs;
        sincospi(2.0 * (double)m / (double)L, &sn, &cs);
        tw[m] = make_double2(cs, -sn);
    }
}

// Element j of a workgroup's tile: line b, index i along the axis, and its
// position in the L^3 array.  Along x the tile is B consecutive rows (one
// contiguous run); along y (z) it is B consecutive x of one z (y), so that a
// wave reads runs of B consecutive elements.
template <int LOG2L, int AXIS>
__device__ __forceinline__ void fft_element(int w, int j, int &b, int &i, size_t &pos)
{
    using S = FftShape<LOG2L>;
    constexpr int L = S::L;
    if constexpr (AXIS == 0) {
        b = j >> LOG2L;
        i = j & (L - 1);
        pos = (size_t)w * S::B * L + (size_t)j;
    } else {
        b = j & (S::B - 1);
        i = j >> S::LOG2B;
        const int x = ((w & (L / S::B - 1)) << S::LOG2B) + b, o = w >> (LOG2L - S::LOG2B);
        pos = AXIS == 1 ? ((size_t)o * L + (size_t)i) * L + (size_t)x : ((size_t)i * L + (size_t)o) * L + (size_t)x;
    }
}

// Passes kFftFwdBitsX .. kFftInvY, one tile per workgroup: L^2 / B tiles,
// except kFftInvY, which needs only the planes z <= L/2 ((L/2 + 1) L / B
// tiles; kFftSquareZ stores only those): the autocorrelation is even, A(-r)
// = A(r), so the shells follow from half of it (fft_bin_kernel).
template <int LOG2L, int OP>
__global__ __launch_bounds__(kFftThreads) void fft_pass_kernel(FftArgs a)
{
    using S = FftShape<LOG2L>;
    constexpr int L = S::L, B = S::B, TILE = B * L;
    constexpr int AXIS = OP == kFftFwdBitsX ? 0 : (OP == kFftSquareZ ? 2 : 1);
    static_assert(OP != kFftInvBinX, "the last pass is fft_bin_kernel");
    __shared__ double2 s[B * S::LP];
    __shared__ double2 tw[L / 2];
    const int tid = (int)threadIdx.x, w = (int)blockIdx.x;

    fft_twiddles<LOG2L>(tw, tid);
    for (int j = tid; j < TILE; j += kFftThreads) {
        int b, i;
        size_t pos;
        fft_element<LOG2L, AXIS>(w, j, b, i, pos);
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
        fft_lines<LOG2L, B, false>(s, tw, tid);
    } else if constexpr (OP == kFftSquareZ) {
        fft_lines<LOG2L, B, false>(s, tw, tid);
        for (int j = tid; j < TILE; j += kFftThreads) {
            double2 *p = s + (j >> LOG2L) * S::LP + (j & (L - 1));
            const double2 v = *p;
            *p = make_double2(v.x * v.x + v.y * v.y, 0.0);
        }
        __syncthreads();
        fft_lines<LOG2L, B, true>(s, tw, tid);
    } else {
        fft_lines<LOG2L, B, true>(s, tw, tid);
    }

    for (int j = tid; j < TILE; j += kFftThreads) {
        int b, i;
        size_t pos;
        fft_element<LOG2L, AXIS>(w, j, b, i, pos);
        if (OP == kFftSquareZ && i > L / 2) continue;
        a.z[pos] = s[b * S::LP + i];
    }
}

constexpr int kFftBinY = 4;  // y values per workgroup of the last pass

// The last pass, on the planes z = 0 .. L/2: a workgroup takes kFftBinY
// values y <= L/2 of one z and, for each, the rows y and L - y (one row if y
// is 0 or L/2), transforms them along x (DIT), and for every |x| = i <= L/2
// adds the rounded sums at x = +-i of both rows to the shell i^2 + y^2 + z^2
// (these are the minimum images) in one atomic.  A row (y, z) and the row
// (L - y, L - z) hold A(x, y, z) and A(-x, y, z), so for 0 < z < L/2 the
// sums count twice for the planes L - z that are not transformed.
template <int LOG2L>
__global__ __launch_bounds__(kFftThreads) void fft_bin_kernel(FftArgs a)
{
    constexpr int L = 1 << LOG2L, H = L / 2, LP = L + 1, NL = 2 * kFftBinY;
    constexpr int YB = (H + 1 + kFftBinY - 1) / kFftBinY;  // workgroups per plane
    __shared__ double2 s[NL * LP];
    __shared__ double2 tw[H];
    const int tid = (int)threadIdx.x, w = (int)blockIdx.x;
    const int z = w / YB, y0 = (w - z * YB) * kFftBinY;

    fft_twiddles<LOG2L>(tw, tid);
    // line 2j: row (y0 + j, z); line 2j + 1: row (L - y0 - j, z) if 0 < y0 + j < L/2
    for (int j = tid; j < NL * L; j += kFftThreads) {
        const int line = j >> LOG2L, x = j & (L - 1), y = y0 + (line >> 1);
        const bool mirror = (line & 1) != 0;
        double2 v = make_double2(0.0, 0.0);
        if (y <= H && (!mirror || (y != 0 && y != H)))
            v = a.z[((size_t)z * L + (size_t)(mirror ? L - y : y)) * L + (size_t)x];
        s[line * LP + x] = v;
    }
    __syncthreads();
    fft_lines<LOG2L, NL, true>(s, tw, tid);

    const long long weight = (z == 0 || z == H) ? 1 : 2;
    for (int t = tid; t < kFftBinY * (H + 1); t += kFftThreads) {
        const int j = t / (H + 1), i = t - j * (H + 1), y = y0 + j;
        if (y > H) continue;
        const int k = i * i + y * y + z * z;
        if (k >= a.n_shells) continue;
        long long sum = 0;
        bool bad = false;
#pragma unroll
        for (int e = 0; e < 4; ++e) {  // bit 0: x -> L - x, bit 1: y -> L - y
            if ((e & 1) && (i == 0 || i == H)) continue;
            if ((e & 2) && (y == 0 || y == H)) continue;
            const double v = ldexp(s[(2 * j + (e >> 1)) * LP + ((e & 1) ? L - i : i)].x, -3 * LOG2L);
            const double r = rint(v);
            bad |= !(fabs(v - r) <= 0.25);  // NaN included
            sum += (long long)r;
        }
        if (bad) atomicOr(a.err, 1u);
        atomicAdd(a.shells + k, (unsigned long long)(sum * weight));
    }
}

}  // namespace ea
