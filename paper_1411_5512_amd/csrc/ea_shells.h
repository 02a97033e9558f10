// ea_shells.h -- full-vector C4 (eq. 3 over every displacement r, summed by
// minimum-image distance shells) for lattices up to L = 256, and for the
// configurations of the batched and multispin-coded forms.
//
// Both work on the dense overlap rows of ea_kernels.h (dense_q_kernel): for
// each row (y, z) the L sites' q = S_0 xor S_1 in natural x order, twice
// (bits [0, L) and [L, 2L)), in 2 NW 64-bit words, NW = ceil(L / 64), so that
// the row shifted cyclically by rx is the window of L bits starting at bit rx.
#pragma once

#include "ea_kernels.h"
#include "ea_msc_kernels.h"

namespace ea {

// Dense overlap rows of one sample of a multispin batch: sample m of word set
// gi, whose site (x, y, z) is bit k M + m of the word at reduced position
// (x >> 1, y, z - k Lz), k = z / Lz, of colour (x + y + z) & 1.  One thread
// per (row, word of the doubled row).
__global__ __launch_bounds__(256) void msc_dense_q_kernel(MscLattice lat, MscGeom g, int M, int gi, int m, int dw,
                                                          unsigned long long *qd)
{
    const int L = g.L;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= L * L * dw) return;
    const int row = gid / dw;
    const int j = gid - row * dw;
    const int y = row % L, z = row / L;
    const int k = z / g.Lz, zr = z - k * g.Lz;
    const int bit = k * M + m;
    const uint32_t *s0 = lat.spins + msc_spin_plane(g, gi, 0, 0), *s1 = lat.spins + msc_spin_plane(g, gi, 1, 0);
    unsigned long long bits = 0;
    for (int b = 0; b < 64; ++b) {
        const int gbit = 64 * j + b;
        if (gbit >= 2 * L) break;
        const int x = gbit % L;
        const int c = (x + y + z) & 1;
        const size_t word = (size_t)c * g.P + (size_t)(x >> 1) + (size_t)g.R * ((size_t)y + (size_t)L * zr);
        bits |= (unsigned long long)(((s0[word] ^ s1[word]) >> bit) & 1u) << b;
    }
    qd[gid] = bits;
}

constexpr int kShellChunk = 16;  // displacements rx per workgroup; divides 64

// Workgroup (chunk of kShellChunk displacements rx, ry + L rz): every thread
// takes source rows with a stride, holds the source row (NW words) and the
// NW + 1 words of the partner row at (y + ry, z + rz) from word rx0 / 64 on
// (the same for every rx of the chunk, as the chunk does not cross a 64-bit
// boundary), counts the sites where q differs from q at x + r, the workgroup
// adds the counts, and N - 2 * count = sum_x q(x) q(x + r) goes to the shell
// of r.  Any NW (L <= 64 NW).
template <int NW>
__global__ __launch_bounds__(256) void c4_shell_rows_kernel(const unsigned long long *qd, int L, int n_shells,
                                                            unsigned long long *shells)
{
    constexpr int DW = 2 * NW;
    __shared__ unsigned int part[kShellChunk][256 / 64];
    const int rx0 = blockIdx.x * kShellChunk;
    const int ry = (int)(blockIdx.y % (unsigned)L), rz = (int)(blockIdx.y / (unsigned)L);
    const int kyz = min_image_sq(ry, L) + min_image_sq(rz, L);
    int kmin = 1 << 30;
    for (int i = 0; i < kShellChunk; ++i)
        if (rx0 + i < L) kmin = min(kmin, kyz + min_image_sq(rx0 + i, L));
    if (kmin >= n_shells) return;  // whole workgroup: no barrier passed yet
    const int w0 = rx0 >> 6;
    const int tail = L - 64 * (NW - 1);  // bits used in the last word of a row
    const unsigned long long last_mask = tail == 64 ? ~0ull : ((1ull << tail) - 1ull);
    unsigned int cnt[kShellChunk];
#pragma unroll
    for (int i = 0; i < kShellChunk; ++i) cnt[i] = 0;
    const int rows = L * L;
    for (int row = (int)threadIdx.x; row < rows; row += (int)blockDim.x) {
        const int y = row % L, z = row / L;
        const int prow = (y + ry) % L + L * ((z + rz) % L);
        unsigned long long src[NW], par[NW + 1];
#pragma unroll
        for (int j = 0; j < NW; ++j) src[j] = qd[(size_t)row * DW + j];
#pragma unroll
        for (int j = 0; j <= NW; ++j) par[j] = qd[(size_t)prow * DW + w0 + j];  // w0 + NW < DW
#pragma unroll
        for (int i = 0; i < kShellChunk; ++i) {
            const int rx = rx0 + i;  // uniform across the workgroup
            if (rx >= L) break;
            const int off = rx & 63;
            unsigned int c = 0;
#pragma unroll
            for (int j = 0; j < NW; ++j) {
                const unsigned long long win = off ? ((par[j] >> off) | (par[j + 1] << (64 - off))) : par[j];
                unsigned long long d = src[j] ^ win;
                if (j == NW - 1) d &= last_mask;
                c += (unsigned int)__popcll(d);
            }
            cnt[i] += c;
        }
    }
#pragma unroll
    for (int i = 0; i < kShellChunk; ++i) {
        const uint32_t v = wave_sum(cnt[i]);
        if ((threadIdx.x & 63) == 0) part[i][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < kShellChunk) {
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

}  // namespace ea
