// ea_probe.hip -- instruction-rate probes behind the integer-ALU roofline of
// the update (built as libea_probe.so, separate from the library; only the
// benchmark loads it).
//
// The roofline prices a Philox4x32-10 block (Salmon et al., SC'11) at
// 10 rounds x (2 32x32->64-bit multiplies + 2 three-way XORs) = 40 lane-ops
// for 4 random words, i.e. it counts a 64-bit-product multiply-add
// (v_mad_u64_u32) and a three-input bitwise op (v_bitop3_b32) as one VALU
// issue each.  These kernels measure the sustained lane rate of each
// instruction and of whole Philox blocks on the device, for comparison with
// 256 CUs x 4 SIMDs x 16 lanes x clock.
//
// Every thread runs 8 independent chains (enough to cover the pipeline
// latency with a few waves per SIMD) for `iters` iterations of 16 steps; the
// results are folded into one word per thread and stored, so that nothing is
// dead code.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;
constexpr int kSteps = 16;

__global__ __launch_bounds__(256) void mad_u64_probe(uint32_t iters, uint32_t seed, uint32_t *sink)
{
    uint64_t m[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        m[c] = ((uint64_t)(seed + blockIdx.x + (uint32_t)c) << 32) | (seed + threadIdx.x * 7u + (uint32_t)c);
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
#pragma unroll
            for (int c = 0; c < kChains; ++c)  // one v_mad_u64_u32: hi(m) x constant + m
                m[c] = (uint64_t)(uint32_t)(m[c] >> 32) * 0xD2511F53u + m[c];
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= (uint32_t)m[c] ^ (uint32_t)(m[c] >> 32);
    sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// The three-input op with a non-linear table (bitwise majority), so that
// the compiler cannot fold a chain of them; its issue rate does not depend
// on the table.
__global__ __launch_bounds__(256) void bitop3_probe(uint32_t iters, uint32_t seed, uint32_t *sink)
{
    uint32_t x[kChains], k[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        x[c] = seed + threadIdx.x * 5u + (uint32_t)c * 0x01010101u;
        k[c] = (seed ^ threadIdx.x) + (uint32_t)c * 0x9E3779B9u;
    }
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_bitop3_b32(x[c], x[c ^ 1], k[c], 0xE8);
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= x[c];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// Whole Philox4x32-10 blocks, two interleaved per thread, counter varied per
// iteration: 40 lane-ops per block by the roofline's count.
__global__ __launch_bounds__(256) void philox_probe(uint32_t iters, uint32_t seed, uint32_t *sink)
{
    uint32_t acc = 0;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t i = 0; i < iters; ++i) {
        uint32_t a0 = i, a1 = tid, a2 = 0x100u, a3 = seed;
        uint32_t b0 = i, b1 = tid ^ 0x80000000u, b2 = 0x100u, b3 = seed;
        uint32_t k0 = seed, k1 = ~seed;
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            const uint64_t ma0 = (uint64_t)a0 * 0xD2511F53u, mb0 = (uint64_t)b0 * 0xD2511F53u;
            const uint64_t ma2 = (uint64_t)a2 * 0xCD9E8D57u, mb2 = (uint64_t)b2 * 0xCD9E8D57u;
            const uint32_t ya0 = __builtin_amdgcn_bitop3_b32((uint32_t)(ma2 >> 32), a1, k0, 0x96);
            const uint32_t yb0 = __builtin_amdgcn_bitop3_b32((uint32_t)(mb2 >> 32), b1, k0, 0x96);
            const uint32_t ya2 = __builtin_amdgcn_bitop3_b32((uint32_t)(ma0 >> 32), a3, k1, 0x96);
            const uint32_t yb2 = __builtin_amdgcn_bitop3_b32((uint32_t)(mb0 >> 32), b3, k1, 0x96);
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
        acc ^= a0 ^ a1 ^ a2 ^ a3 ^ b0 ^ b1 ^ b2 ^ b3;
    }
    sink[tid] = acc;
}

}  // namespace

extern "C" {

// Run probe `kind` (0: v_mad_u64_u32, 1: v_bitop3_b32, 2: Philox4x32-10
// blocks) on `blocks` workgroups of 256 threads for `iters`
// iterations; *ms receives the event-timed duration of the timed launch
// (after one untimed warm-up launch) and *ops the lane-operations it counts
// (instructions x lanes; 40 per Philox block).  Returns 0, or the HIP error.
int ea_probe_alu(int kind, int blocks, unsigned iters, double *ms, double *ops)
{
    if (kind < 0 || kind > 2 || blocks < 1 || !ms || !ops) return -1;
    uint32_t *sink = nullptr;
    hipError_t e = hipMalloc((void **)&sink, (size_t)blocks * 256 * 4);
    if (e != hipSuccess) return (int)e;
    hipEvent_t a = nullptr, b = nullptr;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    double per_iter = 0.0;
    for (int rep = 0; rep < 2; ++rep) {
        (void)hipEventRecord(a, 0);
        switch (kind) {
        case 0:
            hipLaunchKernelGGL(mad_u64_probe, dim3(blocks), dim3(256), 0, 0, iters, 12345u, sink);
            per_iter = kChains * kSteps;
            break;
        case 1:
            hipLaunchKernelGGL(bitop3_probe, dim3(blocks), dim3(256), 0, 0, iters, 12345u, sink);
            per_iter = kChains * kSteps;
            break;
        default:
            hipLaunchKernelGGL(philox_probe, dim3(blocks), dim3(256), 0, 0, iters, 12345u, sink);
            per_iter = 2 * 40;
            break;
        }
        (void)hipEventRecord(b, 0);
    }
    e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(sink);
    if (e != hipSuccess) return (int)e;
    *ms = t;
    *ops = per_iter * (double)iters * (double)blocks * 256.0;
    return 0;
}

}  // extern "C"
