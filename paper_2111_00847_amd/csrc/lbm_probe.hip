// lbm_probe.hip -- HBM streaming probes: the read, write and copy rates one
// MI355X sustains, the measured ceiling that the step kernels' bandwidth is
// set against (next to the nominal 8 TB/s).
//
// Each probe is a grid-stride loop over 16-byte elements (one u32x4 per lane
// and iteration, coalesced), with a grid of `blocks` workgroups of 256
// threads: the sweep over grid sizes finds the rate of the memory system, not
// of one launch shape.  Stores are non-temporal when `nt` is set (a stream
// larger than the 256 MB last-level cache gains nothing from keeping it).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/lbm.h"

namespace lbm {

int hip_fail(hipError_t e);

constexpr int PROBE_THREADS = 256;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // one 16-byte element

// read: every element is loaded and folded into a per-thread value, written
// once per thread so that the loads cannot be dropped.
__global__ __launch_bounds__(PROBE_THREADS) void k_probe_read(const u32x4* __restrict__ src, size_t n,
                                                              uint32_t* __restrict__ sink) {
    const size_t stride = (size_t)gridDim.x * PROBE_THREADS;
    size_t i = (size_t)blockIdx.x * PROBE_THREADS + threadIdx.x;
    uint32_t acc = 0;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const u32x4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        const u32x4 e = (a ^ b) ^ (c ^ d);
        acc ^= (e.x ^ e.y) ^ (e.z ^ e.w);
    }
    for (; i < n; i += stride) {
        const u32x4 a = src[i];
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    sink[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = acc;
}

template <bool NT>
__global__ __launch_bounds__(PROBE_THREADS) void k_probe_write(u32x4* __restrict__ dst, size_t n, uint32_t v) {
    const size_t stride = (size_t)gridDim.x * PROBE_THREADS;
    const u32x4 w = {v, v + 1, v + 2, v + 3};
    for (size_t i = (size_t)blockIdx.x * PROBE_THREADS + threadIdx.x; i < n; i += stride) {
        if (NT) __builtin_nontemporal_store(w, dst + i);
        else dst[i] = w;
    }
}

template <bool NT>
__global__ __launch_bounds__(PROBE_THREADS) void k_probe_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                              size_t n) {
    const size_t stride = (size_t)gridDim.x * PROBE_THREADS;
    size_t i = (size_t)blockIdx.x * PROBE_THREADS + threadIdx.x;
    for (; i + stride < n; i += 2 * stride) {
        const u32x4 a = src[i], b = src[i + stride];
        if (NT) {
            __builtin_nontemporal_store(a, dst + i);
            __builtin_nontemporal_store(b, dst + i + stride);
        } else {
            dst[i] = a;
            dst[i + stride] = b;
        }
    }
    for (; i < n; i += stride) {
        if (NT) __builtin_nontemporal_store(src[i], dst + i);
        else dst[i] = src[i];
    }
}

}  // namespace lbm

using namespace lbm;

extern "C" int lbm_bandwidth_probe(int32_t kind, void* dst, const void* src, size_t bytes, int32_t blocks,
                                   int32_t nt, void* stream) {
    if (kind < 0 || kind > 2) return LBM_E_PARAM;
    if (blocks < 1 || bytes < 16 || bytes % 16) return LBM_E_SIZE;
    if (((uintptr_t)dst | (uintptr_t)src) % 16) return LBM_E_SIZE;
    if ((kind != 1 && !src) || !dst) return LBM_E_NULL;
    hipStream_t s = (hipStream_t)stream;
    const size_t n = bytes / 16;
    if (kind == 0)
        k_probe_read<<<blocks, PROBE_THREADS, 0, s>>>(static_cast<const u32x4*>(src), n, static_cast<uint32_t*>(dst));
    else if (kind == 1 && nt)
        k_probe_write<true><<<blocks, PROBE_THREADS, 0, s>>>(static_cast<u32x4*>(dst), n, 0x9e3779b9u);
    else if (kind == 1)
        k_probe_write<false><<<blocks, PROBE_THREADS, 0, s>>>(static_cast<u32x4*>(dst), n, 0x9e3779b9u);
    else if (nt)
        k_probe_copy<true><<<blocks, PROBE_THREADS, 0, s>>>(static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n);
    else
        k_probe_copy<false><<<blocks, PROBE_THREADS, 0, s>>>(static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : hip_fail(e);
}
