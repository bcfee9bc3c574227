// probe.hip -- streaming bandwidth probe of the device (read-only, write-only
// and copy kernels over one buffer), used to state what HBM bandwidth the
// stencil kernels can reach on this part and to calibrate the hardware
// traffic counters (a probe of known size reads FETCH_SIZE / WRITE_SIZE for a
// known number of bytes).
//
// Each kernel walks the buffer in 16-byte elements with a grid-stride loop,
// four independent elements in flight per thread per iteration; the grid is a
// fixed multiple of the compute units so every CU streams.  The read kernel
// folds what it reads with XOR into one 16-byte word per block, written to
// dst (so nothing it reads is dead); the write kernel stores a pattern.
#include "dpml.h"

#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 4;

template <bool NT>
__device__ __forceinline__ uint4 probe_ld(const uint4 *p)
{
    if constexpr (NT) {
        uint4 v;
        v.x = __builtin_nontemporal_load(&p->x);
        v.y = __builtin_nontemporal_load(&p->y);
        v.z = __builtin_nontemporal_load(&p->z);
        v.w = __builtin_nontemporal_load(&p->w);
        return v;
    } else {
        return *p;
    }
}

template <bool NT>
__device__ __forceinline__ void probe_st(uint4 *p, uint4 v)
{
    if constexpr (NT) {
        __builtin_nontemporal_store(v.x, &p->x);
        __builtin_nontemporal_store(v.y, &p->y);
        __builtin_nontemporal_store(v.z, &p->z);
        __builtin_nontemporal_store(v.w, &p->w);
    } else {
        *p = v;
    }
}

__device__ __forceinline__ uint4 xor4(uint4 a, uint4 b)
{
    return make_uint4(a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w);
}

template <bool NT>
__global__ void __launch_bounds__(kProbeThreads) k_probe_read(const uint4 *__restrict__ src, int64_t nv,
                                                              uint4 *__restrict__ partial)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    uint4 acc = make_uint4(0, 0, 0, 0);
    for (; i + (kProbeUnroll - 1) * stride < nv; i += kProbeUnroll * stride) {
        uint4 v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) v[u] = probe_ld<NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) acc = xor4(acc, v[u]);
    }
    for (; i < nv; i += stride) acc = xor4(acc, probe_ld<NT>(src + i));
    // fold the block's words through LDS, one store per block
    __shared__ uint4 red[kProbeThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kProbeThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = xor4(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

template <bool NT>
__global__ void __launch_bounds__(kProbeThreads) k_probe_write(uint4 *__restrict__ dst, int64_t nv, uint32_t pattern)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    const uint4 v = make_uint4(pattern, pattern + 1, pattern + 2, pattern + 3);
    for (; i + (kProbeUnroll - 1) * stride < nv; i += kProbeUnroll * stride) {
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) probe_st<NT>(dst + i + u * stride, v);
    }
    for (; i < nv; i += stride) probe_st<NT>(dst + i, v);
}

template <bool NT>
__global__ void __launch_bounds__(kProbeThreads) k_probe_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                                              int64_t nv)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    for (; i + (kProbeUnroll - 1) * stride < nv; i += kProbeUnroll * stride) {
        uint4 v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) v[u] = probe_ld<NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) probe_st<NT>(dst + i + u * stride, v[u]);
    }
    for (; i < nv; i += stride) probe_st<NT>(dst + i, probe_ld<NT>(src + i));
}

}  // namespace

extern "C" int dpml_bandwidth_probe(int32_t kind, void *dst, const void *src, size_t bytes, int32_t blocks_per_cu,
                                    int32_t reps, void *stream, double *ms_per_rep)
{
    const int op = kind & 3;
    const bool nt = (kind & DPML_PROBE_NONTEMPORAL) != 0;
    if (op > DPML_PROBE_COPY || (kind & ~(3 | DPML_PROBE_NONTEMPORAL)) || reps < 1 || !ms_per_rep) return DPML_EINVAL;
    if (bytes == 0 || bytes % 16 != 0) return DPML_EINVAL;
    if ((op != DPML_PROBE_WRITE && !src) || !dst) return DPML_EINVAL;
    if (((uintptr_t)dst | (uintptr_t)src) % 16 != 0) return DPML_EINVAL;
    if (blocks_per_cu < 1 || blocks_per_cu > 64) return DPML_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DPML_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return DPML_EHIP;
    const int64_t nv = (int64_t)(bytes / 16);
    int64_t grid = (int64_t)cus * blocks_per_cu;
    const int64_t need = (nv + kProbeThreads - 1) / kProbeThreads;
    if (grid > need) grid = need;
    if (op == DPML_PROBE_READ && grid > (int64_t)DPML_PROBE_MAX_BLOCKS) grid = DPML_PROBE_MAX_BLOCKS;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return DPML_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return DPML_EHIP;
    }
    int rc = DPML_OK;
    const dim3 g((unsigned)grid), b(kProbeThreads);
    if (hipEventRecord(e0, st) != hipSuccess) rc = DPML_EHIP;
    for (int r = 0; r < reps && rc == DPML_OK; ++r) {
        if (op == DPML_PROBE_READ) {
            if (nt) hipLaunchKernelGGL(k_probe_read<true>, g, b, 0, st, (const uint4 *)src, nv, (uint4 *)dst);
            else hipLaunchKernelGGL(k_probe_read<false>, g, b, 0, st, (const uint4 *)src, nv, (uint4 *)dst);
        } else if (op == DPML_PROBE_WRITE) {
            if (nt) hipLaunchKernelGGL(k_probe_write<true>, g, b, 0, st, (uint4 *)dst, nv, (uint32_t)r);
            else hipLaunchKernelGGL(k_probe_write<false>, g, b, 0, st, (uint4 *)dst, nv, (uint32_t)r);
        } else {
            if (nt) hipLaunchKernelGGL(k_probe_copy<true>, g, b, 0, st, (uint4 *)dst, (const uint4 *)src, nv);
            else hipLaunchKernelGGL(k_probe_copy<false>, g, b, 0, st, (uint4 *)dst, (const uint4 *)src, nv);
        }
        if (hipGetLastError() != hipSuccess) rc = DPML_EHIP;
    }
    if (rc == DPML_OK && hipEventRecord(e1, st) != hipSuccess) rc = DPML_EHIP;
    if (rc == DPML_OK && hipEventSynchronize(e1) != hipSuccess) rc = DPML_EHIP;
    float ms = 0.f;
    if (rc == DPML_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = DPML_EHIP;
    if (rc == DPML_OK) *ms_per_rep = (double)ms / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}
