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
// so no pass permutes its data.  The sums are integers of magnitude <= N and
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
// x + rounding and shell sums.
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

// One radix-2 stage of span h = 2^s on every line of the tile.  DIF: (a, b)
// -> (a + b, (a - b) w); DIT: t = b w, (a, b) -> (a + t, a - t); w =
// exp(-+2 pi i pos / 2h) from the table tw[m] = exp(-2 pi i m / L).
template <int LOG2L, bool DIT>
__device__ __forceinline__ void fft_stage(double2 *s, const double2 *tw, int st, int tid)
{
    using S = FftShape<LOG2L>;
    constexpr int H = S::L / 2;
    const int h = 1 << st;
    for (int t = tid; t < S::B * H; t += kFftThreads) {
        const int b = t >> (LOG2L - 1), kk = t & (H - 1);
        const int pos = kk & (h - 1);
        const int i0 = ((kk >> st) << (st + 1)) | pos;
        double2 w = tw[pos << (LOG2L - 1 - st)];
        double2 *p0 = s + b * S::LP + i0, *p1 = p0 + h;
        const double2 a = *p0, c = *p1;
        if constexpr (DIT) {
            w.y = -w.y;
            const double2 u = cmul(c, w);
            *p0 = make_double2(a.x + u.x, a.y + u.y);
            *p1 = make_double2(a.x - u.x, a.y - u.y);
        } else {
            *p0 = make_double2(a.x + c.x, a.y + c.y);
            *p1 = cmul(make_double2(a.x - c.x, a.y - c.y), w);
        }
    }
}

template <int LOG2L, bool DIT>
__device__ __forceinline__ void fft_lines(double2 *s, const double2 *tw, int tid)
{
    if constexpr (DIT) {
        for (int st = 0; st < LOG2L; ++st) {
            fft_stage<LOG2L, true>(s, tw, st, tid);
            __syncthreads();
        }
    } else {
        for (int st = LOG2L - 1; st >= 0; --st) {
            fft_stage<LOG2L, false>(s, tw, st, tid);
            __syncthreads();
        }
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

// One pass (FftOp) over the L^2 / B tiles, one per workgroup.
template <int LOG2L, int OP>
__global__ __launch_bounds__(kFftThreads) void fft_pass_kernel(FftArgs a)
{
    using S = FftShape<LOG2L>;
    constexpr int L = S::L, B = S::B, TILE = B * L;
    constexpr int AXIS = OP == kFftFwdBitsX || OP == kFftInvBinX ? 0 : (OP == kFftSquareZ ? 2 : 1);
    __shared__ double2 s[B * S::LP];
    __shared__ double2 tw[L / 2];
    const int tid = (int)threadIdx.x, w = (int)blockIdx.x;

    for (int m = tid; m < L / 2; m += kFftThreads) {
        double sn, cs;
        sincospi(2.0 * (double)m / (double)L, &sn, &cs);
        tw[m] = make_double2(cs, -sn);
    }
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
        fft_lines<LOG2L, false>(s, tw, tid);
    } else if constexpr (OP == kFftSquareZ) {
        fft_lines<LOG2L, false>(s, tw, tid);
        for (int j = tid; j < TILE; j += kFftThreads) {
            double2 *p = s + (j >> LOG2L) * S::LP + (j & (L - 1));
            const double2 v = *p;
            *p = make_double2(v.x * v.x + v.y * v.y, 0.0);
        }
        __syncthreads();
        fft_lines<LOG2L, true>(s, tw, tid);
    } else {
        fft_lines<LOG2L, true>(s, tw, tid);
    }

    if constexpr (OP != kFftInvBinX) {
        for (int j = tid; j < TILE; j += kFftThreads) {
            int b, i;
            size_t pos;
            fft_element<LOG2L, AXIS>(w, j, b, i, pos);
            a.z[pos] = s[b * S::LP + i];
        }
    } else {
        // rows w B .. w B + B - 1: row y + L z holds N sum_x q(x) q(x + r) at
        // r = (i, y, z).  Displacements i and L - i share a shell: one atomic
        // for both.
        constexpr int HALF = L / 2 + 1;
        for (int t = tid; t < B * HALF; t += kFftThreads) {
            const int b = t / HALF, i = t - b * HALF;
            const int row = w * B + b, y = row & (L - 1), z = row >> LOG2L;
            const int my = y < L - y ? y : L - y, mz = z < L - z ? z : L - z;
            const int k = i * i + my * my + mz * mz;
            if (k >= a.n_shells) continue;
            long long sum = 0;
            bool bad = false;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                if (e == 1 && (i == 0 || i == L / 2)) break;
                const double v = ldexp(s[b * S::LP + (e ? L - i : i)].x, -3 * LOG2L);
                const double r = rint(v);
                bad |= !(fabs(v - r) <= 0.25);  // NaN included
                sum += (long long)r;
            }
            if (bad) atomicOr(a.err, 1u);
            atomicAdd(a.shells + k, (unsigned long long)sum);
        }
    }
}

}  // namespace ea
