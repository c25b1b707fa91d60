// Instruction-rate microbenchmarks for the operations CLS tracking is made of.
//
// Each kernel runs NCHAIN independent dependency chains per lane; a chain
// applies one operation per iteration. With enough waves in flight the
// measured rate is the issue throughput of the operation (wave64 lane-ops per
// second), to compare with the full-rate VALU peak of
// 256 CUs x 64 lanes x clock. Results are written to memory so nothing is
// optimized away. Exposed through a small C function for the Python runner.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace {

constexpr int NCHAIN = 8;

enum Op : int {
    OP_FMA_F32 = 0, OP_MAD_U64_U32, OP_MUL_HI_U32, OP_LOG_F32, OP_SIN_F32, OP_SQRT_F32, OP_RCP_F32,
    OP_FMA_F64, OP_BITOP3, OP_LOG_F64, OP_SINCOS_F64, OP_SQRT_F64, OP_DIV_F64, OP_PHILOX,
    OP_LDS_ADD_F64, OP_COUNT
};

template <int OP>
__global__ void __launch_bounds__(256) bench_kernel(uint32_t *out, int iters, uint32_t seed)
{
    __shared__ double lds[1024];
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (OP == OP_LDS_ADD_F64) {
        for (int i = threadIdx.x; i < 1024; i += blockDim.x) lds[i] = 0.0;
        __syncthreads();
    }
    float f[NCHAIN];
    double d[NCHAIN];
    uint32_t u[NCHAIN];
#pragma unroll
    for (int c = 0; c < NCHAIN; ++c) {
        u[c] = tid * 2654435761u + (uint32_t)c * 40503u + seed;
        f[c] = 1.0f + (float)(u[c] & 0xFFFF) * 1e-5f;
        d[c] = 1.0 + (double)(u[c] & 0xFFFF) * 1e-5;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < NCHAIN; ++c) {
            if (OP == OP_FMA_F32) f[c] = __builtin_fmaf(f[c], 0.999f, 0.001f);
            if (OP == OP_MAD_U64_U32) {
                const uint64_t p = (uint64_t)u[c] * 0xD2511F53u + (uint64_t)c;
                u[c] = (uint32_t)(p >> 32) ^ (uint32_t)p;
            }
            if (OP == OP_MUL_HI_U32) u[c] = __umulhi(u[c], 0xCD9E8D57u) + 1u;
            if (OP == OP_LOG_F32) f[c] = __builtin_amdgcn_logf(f[c]) + 1.0f;
            if (OP == OP_SIN_F32) f[c] = __builtin_amdgcn_sinf(f[c]) + 0.5f;
            if (OP == OP_SQRT_F32) f[c] = __builtin_amdgcn_sqrtf(f[c]) + 0.5f;
            if (OP == OP_RCP_F32) f[c] = __builtin_amdgcn_rcpf(f[c]) + 0.5f;
            if (OP == OP_FMA_F64) d[c] = __builtin_fma(d[c], 0.999, 0.001);
            if (OP == OP_BITOP3) u[c] = __builtin_amdgcn_bitop3_b32(u[c], 0x9E3779B9u + c, tid, 0x96);
            if (OP == OP_LOG_F64) d[c] = log(d[c]) + 1.0;
            if (OP == OP_SINCOS_F64) {
                double s, cs;
                sincos(d[c], &s, &cs);
                d[c] = s + cs + 0.5;
            }
            if (OP == OP_SQRT_F64) d[c] = sqrt(d[c]) + 0.5;
            if (OP == OP_DIV_F64) d[c] = 1.0 / d[c] + 0.5;
            if (OP == OP_PHILOX) {
                const cls::Block5 b = cls::philox_u23((uint32_t)it, (uint32_t)c, (uint64_t)u[c], seed, 7u);
                u[c] = b.k[0] ^ b.k[4];
            }
            if (OP == OP_LDS_ADD_F64) {
                atomicAdd(&lds[(u[c] >> 7) & 1023u], 1.0);
                u[c] = u[c] * 1664525u + 1013904223u;
            }
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < NCHAIN; ++c) acc ^= u[c] ^ __float_as_uint(f[c]) ^ (uint32_t)__double_as_longlong(d[c]);
    if (OP == OP_LDS_ADD_F64) {
        __syncthreads();
        acc ^= (uint32_t)lds[threadIdx.x];
    }
    out[tid] = acc;
}

template <int OP>
hipError_t launch(uint32_t *out, int blocks, int iters, hipStream_t s)
{
    hipLaunchKernelGGL(bench_kernel<OP>, dim3(blocks), dim3(256), 0, s, out, iters, 12345u);
    return hipGetLastError();
}

typedef hipError_t (*LaunchFn)(uint32_t *, int, int, hipStream_t);
const LaunchFn kLaunch[OP_COUNT] = {
    launch<OP_FMA_F32>, launch<OP_MAD_U64_U32>, launch<OP_MUL_HI_U32>, launch<OP_LOG_F32>,
    launch<OP_SIN_F32>, launch<OP_SQRT_F32>, launch<OP_RCP_F32>, launch<OP_FMA_F64>,
    launch<OP_BITOP3>, launch<OP_LOG_F64>, launch<OP_SINCOS_F64>, launch<OP_SQRT_F64>,
    launch<OP_DIV_F64>, launch<OP_PHILOX>, launch<OP_LDS_ADD_F64>};

}  // namespace

// Run operation `op` with `blocks` x 256 threads for `iters` iterations of
// NCHAIN operations per lane; returns the kernel time in ms (negative on error).
extern "C" double clsmb_run(int op, int blocks, int iters)
{
    if (op < 0 || op >= OP_COUNT || blocks < 1 || iters < 1) return -1.0;
    uint32_t *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) return -2.0;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    double ms = -3.0;
    if (kLaunch[op](out, blocks, 4, nullptr) == hipSuccess && hipDeviceSynchronize() == hipSuccess) {
        (void)hipEventRecord(a, nullptr);
        const hipError_t e = kLaunch[op](out, blocks, iters, nullptr);
        (void)hipEventRecord(b, nullptr);
        float f = 0.0f;
        if (e == hipSuccess && hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&f, a, b) == hipSuccess)
            ms = f;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(out);
    return ms;
}

extern "C" int clsmb_chains(void) { return NCHAIN; }
