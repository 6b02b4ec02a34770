// probe.hip -- memory-rate microbenchmarks that bound the engine's kernels
// on one MI355X: random 4- and 8-byte gathers and 4-byte atomics over tables
// sized like the traversal state (L2-, MALL- and HBM-resident), random
// distance rows of 64, 128 and 256 bytes (one wave per row, as the batched
// relaxation reads them), and a stream copy.  Not part of the engine ABI:
// a measurement tool driven by the package's probe module.
//
// Every kernel walks a grid-stride loop over `count` operations; operation i
// touches table entry hash(i) mod entries, so every access is in bounds.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint32_t mix32(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    return (uint32_t)x;
}

__global__ void k_gather4(const uint32_t *t, uint64_t entries, uint64_t count, uint32_t *sink)
{
    uint32_t acc = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        acc += t[mix32(i) % entries];
    if (acc == 0x9e3779b9u) sink[0] = acc;   // keeps the loads live
}

__global__ void k_gather8(const unsigned long long *t, uint64_t entries, uint64_t count, uint32_t *sink)
{
    unsigned long long acc = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        acc ^= t[mix32(i) % entries];
    if (acc == 0x9e3779b97f4a7c15ull) sink[0] = (uint32_t)acc;
}

__global__ void k_atomic4(uint32_t *t, uint64_t entries, uint64_t count)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        atomicMin(t + mix32(i) % entries, (uint32_t)i);
}

// one wave per row of `words` 4-byte words (32: 128 bytes, 64: 256 bytes);
// with `amin` every lane also lowers its word with atomicMin
template <int WORDS>
__global__ void k_rows(uint32_t *t, uint64_t rows, uint64_t count, int amin, uint32_t *sink)
{
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t acc = 0;
    // 16 rows in flight per wave
    for (uint64_t i0 = wave * 16; i0 < count; i0 += waves * 16) {
        uint32_t v[16];
        uint64_t r[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            r[j] = mix32(i0 + j) % rows;
            v[j] = (i0 + j < count && lane < WORDS) ? t[r[j] * WORDS + lane] : 0u;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            acc += v[j];
            if (amin && i0 + j < count && lane < WORDS) atomicMin(t + r[j] * WORDS + lane, v[j] >> 1);
        }
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

// 128-byte rows read as 64 lanes x 2 bytes (one row per wave instruction)
__global__ void k_rows16(const uint16_t *t, uint64_t rows, uint64_t count, uint32_t *sink)
{
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t acc = 0;
    for (uint64_t i0 = wave * 16; i0 < count; i0 += waves * 16) {
        uint32_t v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = (i0 + j < count) ? t[(uint64_t)(mix32(i0 + j) % rows) * 64 + lane] : 0u;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc += v[j];
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

// 64-byte rows read as 64 lanes x 1 byte (one row per wave instruction)
__global__ void k_rows8(const uint8_t *t, uint64_t rows, uint64_t count, uint32_t *sink)
{
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t acc = 0;
    for (uint64_t i0 = wave * 16; i0 < count; i0 += waves * 16) {
        uint32_t v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = (i0 + j < count) ? t[(uint64_t)(mix32(i0 + j) % rows) * 64 + lane] : 0u;
#pragma unroll
        for (int j = 0; j < 16; ++j) acc += v[j];
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

// 128-byte rows read two per wave instruction: lanes 0-31 take one row as
// 32 words, lanes 32-63 the next
__global__ void k_rows_pair(const uint32_t *t, uint64_t rows, uint64_t count, uint32_t *sink)
{
    const int lane = threadIdx.x & 63, half = lane >> 5, w = lane & 31;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t acc = 0;
    for (uint64_t i0 = wave * 16; i0 < count; i0 += waves * 16) {
        uint32_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint64_t i = i0 + 2 * j + half;
            v[j] = (i < count) ? t[(uint64_t)(mix32(i) % rows) * 32 + w] : 0u;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += v[j];
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

// 64-byte rows read four per wave instruction: lanes 16k..16k+15 take row k
// as 16 words; with `amin`, the first lane of each quarter also lowers one
// word of its row (one scattered atomic per row)
__global__ void k_rows_quad(uint32_t *t, uint64_t rows, uint64_t count, int amin, uint32_t *sink)
{
    const int lane = threadIdx.x & 63, quarter = lane >> 4, w = lane & 15;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t acc = 0;
    for (uint64_t i0 = wave * 32; i0 < count; i0 += waves * 32) {
        uint32_t v[8];
        uint64_t r[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint64_t i = i0 + 4 * j + quarter;
            r[j] = mix32(i) % rows;
            v[j] = (i < count) ? t[r[j] * 16 + w] : 0u;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            acc += v[j];
            if (amin && w == 0 && i0 + 4 * j + quarter < count) atomicMin(t + r[j] * 16 + (v[j] & 15u), v[j] >> 1);
        }
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

// 256-byte rows read two per wave instruction: lanes 0-31 take one row as 32
// 8-byte words, lanes 32-63 the next
__global__ void k_rows256_pair(const unsigned long long *t, uint64_t rows, uint64_t count, uint32_t *sink)
{
    const int lane = threadIdx.x & 63, half = lane >> 5, w = lane & 31;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long acc = 0;
    for (uint64_t i0 = wave * 16; i0 < count; i0 += waves * 16) {
        unsigned long long v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint64_t i = i0 + 2 * j + half;
            v[j] = (i < count) ? t[(uint64_t)(mix32(i) % rows) * 32 + w] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += v[j];
    }
    if (acc == 0x9e3779b97f4a7c15ull) sink[0] = (uint32_t)acc;
}

__global__ void k_copy(const uint4 *a, uint4 *b, uint64_t n16)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) b[i] = a[i];
}

__global__ void k_fill(uint32_t *t, uint64_t n, uint32_t v)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) t[i] = v ^ (uint32_t)i;
}

int grid_of(int per_cu)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    }
    return cus * per_cu;
}

}  // namespace

// Each entry point returns the device time in milliseconds of one launch
// (after one untimed warm-up launch), or a negative value on a HIP error.
// Tables are allocated and filled inside; `bytes` is the table size.
extern "C" {

float probe_run(int kind, uint64_t bytes, uint64_t count)
{
    void *t = nullptr, *u = nullptr;
    uint32_t *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = -1.f;
    const int G = grid_of(8);
    if (hipMalloc(&t, bytes) != hipSuccess) return -1.f;
    if (kind == 7 && hipMalloc(&u, bytes) != hipSuccess) {
        (void)hipFree(t);
        return -1.f;
    }
    if (hipMalloc((void **)&sink, 256) != hipSuccess) {
        (void)hipFree(t);
        if (u) (void)hipFree(u);
        return -1.f;
    }
    hipLaunchKernelGGL(k_fill, dim3(G), dim3(256), 0, 0, (uint32_t *)t, bytes / 4, 0x12345u);
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    auto launch = [&]() {
        switch (kind) {
        case 0: hipLaunchKernelGGL(k_gather4, dim3(G), dim3(256), 0, 0, (const uint32_t *)t, bytes / 4, count, sink); break;
        case 1: hipLaunchKernelGGL(k_gather8, dim3(G), dim3(256), 0, 0, (const unsigned long long *)t, bytes / 8, count, sink); break;
        case 2: hipLaunchKernelGGL(k_atomic4, dim3(G), dim3(256), 0, 0, (uint32_t *)t, bytes / 4, count); break;
        case 3: hipLaunchKernelGGL(k_rows<64>, dim3(G), dim3(256), 0, 0, (uint32_t *)t, bytes / 256, count, 0, sink); break;
        case 4: hipLaunchKernelGGL(k_rows<64>, dim3(G), dim3(256), 0, 0, (uint32_t *)t, bytes / 256, count, 1, sink); break;
        case 5: hipLaunchKernelGGL(k_rows<32>, dim3(G), dim3(256), 0, 0, (uint32_t *)t, bytes / 128, count, 0, sink); break;
        case 6: hipLaunchKernelGGL(k_rows<32>, dim3(G), dim3(256), 0, 0, (uint32_t *)t, bytes / 128, count, 1, sink); break;
        case 7: hipLaunchKernelGGL(k_copy, dim3(G), dim3(256), 0, 0, (const uint4 *)t, (uint4 *)u, bytes / 16); break;
        case 8: hipLaunchKernelGGL(k_rows16, dim3(G), dim3(256), 0, 0, (const uint16_t *)t, bytes / 128, count, sink); break;
        case 9: hipLaunchKernelGGL(k_rows_pair, dim3(G), dim3(256), 0, 0, (const uint32_t *)t, bytes / 128, count, sink); break;
        case 10: hipLaunchKernelGGL(k_rows<16>, dim3(G), dim3(256), 0, 0, (uint32_t *)t, bytes / 64, count, 0, sink); break;
        case 11: hipLaunchKernelGGL(k_rows8, dim3(G), dim3(256), 0, 0, (const uint8_t *)t, bytes / 64, count, sink); break;
        case 12: hipLaunchKernelGGL(k_rows_quad, dim3(G), dim3(256), 0, 0, (uint32_t *)t, bytes / 64, count, 0, sink); break;
        case 13: hipLaunchKernelGGL(k_rows_quad, dim3(G), dim3(256), 0, 0, (uint32_t *)t, bytes / 64, count, 1, sink); break;
        case 14: hipLaunchKernelGGL(k_rows256_pair, dim3(G), dim3(256), 0, 0, (const unsigned long long *)t, bytes / 256, count, sink); break;
        default: break;
        }
    };
    if (kind >= 0 && kind <= 14) {
        launch();   // warm-up (and first touch of the tables)
        (void)hipEventRecord(e0, 0);
        launch();
        (void)hipEventRecord(e1, 0);
        if (hipEventSynchronize(e1) == hipSuccess && hipGetLastError() == hipSuccess)
            (void)hipEventElapsedTime(&ms, e0, e1);
        else
            ms = -1.f;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(t);
    if (u) (void)hipFree(u);
    (void)hipFree(sink);
    return ms;
}

}  // extern "C"
