// Roofline calibration for gfx950: issue rate of the 32-bit VALU instructions
// the 64-bit modular arithmetic is built from, and device copy bandwidth.
// Each probe runs eight independent chains of one exact instruction per thread
// (arithmetic inline asm only; no memory access in asm).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#define ITERS 1024
#define CHAIN32(INS)                                                                    \
    __global__ void k_##INS(uint32_t *out, uint32_t m) {                                \
        uint32_t a[8];                                                                  \
        for (int i = 0; i < 8; i++) a[i] = threadIdx.x + i;                             \
        for (int it = 0; it < ITERS; it++) {                                            \
            _Pragma("unroll") for (int i = 0; i < 8; i++)                               \
                asm volatile(#INS " %0, %0, %1" : "+v"(a[i]) : "v"(m));                 \
        }                                                                               \
        uint32_t s = 0;                                                                 \
        for (int i = 0; i < 8; i++) s ^= a[i];                                          \
        out[blockIdx.x * blockDim.x + threadIdx.x] = s;                                 \
    }

CHAIN32(v_add_u32)
CHAIN32(v_mul_lo_u32)
CHAIN32(v_mul_hi_u32)

__global__ void k_v_mad_u64_u32(uint32_t *out, uint32_t m) {
    uint64_t a[8];
    for (int i = 0; i < 8; i++) a[i] = threadIdx.x + i;
    for (int it = 0; it < ITERS; it++) {
#pragma unroll
        for (int i = 0; i < 8; i++)
            asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(a[i]) : "v"(m), "v"(m) : "vcc");
    }
    uint64_t s = 0;
    for (int i = 0; i < 8; i++) s ^= a[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)s;
}

__global__ void k_copy(const uint4 *__restrict__ a, uint4 *__restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

typedef void (*kfn)(uint32_t *, uint32_t);

static double time_ms(kfn k, uint32_t *buf, int blocks, int threads, uint32_t m) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), 0, 0, buf, m);
    (void)hipEventRecord(a, 0);
    for (int r = 0; r < 5; r++) hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), 0, 0, buf, m);
    (void)hipEventRecord(b, 0);
    (void)hipEventSynchronize(b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms / 5;
}

int main() {
    const int blocks = 256 * 32, threads = 256;
    uint32_t *buf = nullptr;
    if (hipMalloc(&buf, (size_t)blocks * threads * 4) != hipSuccess) return 1;
    const double ops = (double)blocks * threads * ITERS * 8;
    struct { const char *name; kfn k; } probes[] = {
        {"v_add_u32", k_v_add_u32}, {"v_mul_lo_u32", k_v_mul_lo_u32},
        {"v_mul_hi_u32", k_v_mul_hi_u32}, {"v_mad_u64_u32", k_v_mad_u64_u32}};
    for (auto &p : probes)
        printf("%-14s %7.2f T lane-instr/s\n", p.name, ops / time_ms(p.k, buf, blocks, threads, 0x9E3779B1u) / 1e9);
    const size_t bytes = (size_t)4 << 30, n = bytes / 16;
    uint4 *x = nullptr, *y = nullptr;
    if (hipMalloc(&x, bytes) != hipSuccess || hipMalloc(&y, bytes) != hipSuccess) return 1;
    (void)hipMemset(x, 1, bytes);
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    hipLaunchKernelGGL(k_copy, dim3(256 * 64), dim3(256), 0, 0, x, y, n);
    (void)hipEventRecord(a, 0);
    for (int r = 0; r < 5; r++) hipLaunchKernelGGL(k_copy, dim3(256 * 64), dim3(256), 0, 0, x, y, n);
    (void)hipEventRecord(b, 0);
    (void)hipEventSynchronize(b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    printf("copy kernel    %7.1f GB/s (read + write of %zu MiB)\n", 2.0 * bytes * 5 / (ms / 1e3) / 1e9, bytes >> 20);
    return 0;
}
