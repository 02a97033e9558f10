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
// 256 CUs x 4 SIMDs x 32 lanes x clock.
//
// A second probe measures the latency of the exchange the slab path makes
// between workgroups on different compute units (ea_probe_exchange).
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

// Whole Philox4x32-10 blocks, NB interleaved per thread (independent
// dependency chains side by side), counter varied per iteration: 40 lane-ops
// per block by the roofline's count.  Counter words 0 and 2 and the key are
// uniform across the wavefront, as in the update.
template <int NB>
__global__ __launch_bounds__(256) void philox_probe(uint32_t iters, uint32_t seed, uint32_t *sink)
{
    uint32_t acc = 0;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t i = 0; i < iters; ++i) {
        uint32_t x0[NB], x1[NB], x2[NB], x3[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            x0[b] = i;
            x1[b] = tid * NB + (uint32_t)b;
            x2[b] = 0x100u;
            x3[b] = seed;
        }
        uint32_t k0 = seed, k1 = ~seed;
#pragma unroll
        for (int r = 0; r < 10; ++r) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const uint64_t m0 = (uint64_t)x0[b] * 0xD2511F53u;
                const uint64_t m2 = (uint64_t)x2[b] * 0xCD9E8D57u;
                const uint32_t y0 = __builtin_amdgcn_bitop3_b32((uint32_t)(m2 >> 32), x1[b], k0, 0x96);
                const uint32_t y2 = __builtin_amdgcn_bitop3_b32((uint32_t)(m0 >> 32), x3[b], k1, 0x96);
                x1[b] = (uint32_t)m2;
                x3[b] = (uint32_t)m0;
                x0[b] = y0;
                x2[b] = y2;
            }
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) acc ^= x0[b] ^ x1[b] ^ x2[b] ^ x3[b];
    }
    sink[tid] = acc;
}

// Exchange latency between two workgroups in the form the slab path uses:
// 64-bit entries {word, epoch} written with agent-scope stores (through to
// the level all XCDs share) and polled with agent-scope loads until the
// epoch matches.  Workgroup 0 and workgroup `partner` (of kXchgBlocks one-wave
// workgroups, dealt to the XCDs in turn) send `words` entries back and forth
// `iters` times, one way per iteration.  Every wait gives up after
// kXchgTimeout ticks of the 100 MHz real-time counter and sets err (2), so
// the kernel always ends; a wrong word sets err (1).
constexpr int kXchgBlocks = 16;
constexpr unsigned long long kXchgTimeout = 100000000ull;  // 1 s

__global__ __launch_bounds__(64) void xchg_probe(int partner, int iters, int words, unsigned long long *buf,
                                                 uint32_t *err, unsigned long long *res, uint32_t *xcc)
{
    uint32_t x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    if (threadIdx.x == 0) xcc[blockIdx.x] = x;
    int me;
    if (blockIdx.x == 0)
        me = 0;
    else if ((int)blockIdx.x == partner)
        me = 1;
    else
        return;
    const int lane = (int)threadIdx.x;
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    for (int i = 0; i < iters; ++i) {
        const int sender = i & 1;
        unsigned long long *b = buf + (size_t)sender * (size_t)words;
        const uint32_t epoch = (uint32_t)i + 1u;
        if (sender == me) {
            for (int j = lane; j < words; j += 64)
                __hip_atomic_store(b + j, ((unsigned long long)epoch << 32) | (uint32_t)(i * 7919 + j),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const unsigned long long start = __builtin_amdgcn_s_memrealtime();
            uint32_t bad = 0;
            for (int j = lane; j < words && !bad; j += 64) {
                unsigned long long v;
                for (;;) {
                    v = __hip_atomic_load(b + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((uint32_t)(v >> 32) == epoch) break;
                    if (__builtin_amdgcn_s_memrealtime() - start > kXchgTimeout) {
                        bad = 2;
                        break;
                    }
                }
                if (!bad && (uint32_t)v != (uint32_t)(i * 7919 + j)) bad = 1;
            }
            if (bad) atomicOr(err, bad);
            if (__any(bad == 2)) break;  // the partner stopped: end
        }
    }
    if (lane == 0) res[me] = __builtin_amdgcn_s_memrealtime() - t0;
}

}  // namespace

extern "C" {

// Run probe `kind` (0: v_mad_u64_u32, 1: v_bitop3_b32, 2: Philox4x32-10
// blocks two at a time, 3: one at a time, 4: four at a time) on `blocks`
// workgroups of 256 threads for `iters` iterations; *ms receives the event-timed duration of the timed launch
// (after one untimed warm-up launch) and *ops the lane-operations it counts
// (instructions x lanes; 40 per Philox block).  Returns 0, or the HIP error.
int ea_probe_alu(int kind, int blocks, unsigned iters, double *ms, double *ops)
{
    if (kind < 0 || kind > 4 || blocks < 1 || !ms || !ops) return -1;
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
        case 2:
            hipLaunchKernelGGL(philox_probe<2>, dim3(blocks), dim3(256), 0, 0, iters, 12345u, sink);
            per_iter = 2 * 40;
            break;
        case 3:
            hipLaunchKernelGGL(philox_probe<1>, dim3(blocks), dim3(256), 0, 0, iters, 12345u, sink);
            per_iter = 40;
            break;
        default:
            hipLaunchKernelGGL(philox_probe<4>, dim3(blocks), dim3(256), 0, 0, iters, 12345u, sink);
            per_iter = 4 * 40;
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

// One-way latency (microseconds) of the slab path's exchange between
// workgroup 0 and workgroup `partner` (1 .. 15), `words` entries (1 .. 1024)
// per message, averaged over `iters` (2 .. 100000) messages; the XCDs the two
// ran on go to xcc[0], xcc[1].  0 on success, 1 on a bad argument, 2 on a
// HIP error, 3 if a word came back wrong or a wait timed out.
int ea_probe_exchange(int partner, int words, int iters, double *one_way_us, uint32_t *xcc_out)
{
    if (partner < 1 || partner >= kXchgBlocks || words < 1 || words > 1024 || iters < 2 || iters > 100000 ||
        !one_way_us || !xcc_out)
        return 1;
    unsigned long long *buf = nullptr, *res = nullptr;
    uint32_t *err = nullptr, *xcc = nullptr;
    hipError_t e = hipMalloc((void **)&buf, 2 * (size_t)words * 8);
    if (e == hipSuccess) e = hipMalloc((void **)&res, 2 * 8);
    if (e == hipSuccess) e = hipMalloc((void **)&err, 4);
    if (e == hipSuccess) e = hipMalloc((void **)&xcc, kXchgBlocks * 4);
    if (e == hipSuccess) e = hipMemset(buf, 0, 2 * (size_t)words * 8);
    if (e == hipSuccess) e = hipMemset(err, 0, 4);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(xchg_probe, dim3(kXchgBlocks), dim3(64), 0, 0, partner, iters, words, buf, err, res, xcc);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    unsigned long long r[2] = {0, 0};
    uint32_t bad = 0, xc[kXchgBlocks] = {};
    if (e == hipSuccess) e = hipMemcpy(r, res, sizeof r, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&bad, err, 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(xc, xcc, sizeof xc, hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    (void)hipFree(res);
    (void)hipFree(err);
    (void)hipFree(xcc);
    if (e != hipSuccess) return 2;
    if (bad) return 3;
    *one_way_us = (double)r[0] * 0.01 / iters;  // 100 MHz ticks
    xcc_out[0] = xc[0];
    xcc_out[1] = xc[partner];
    return 0;
}

}  // extern "C"
