// Bandwidth probes: the practical HBM ceiling the products are measured
// against.  Not part of the method: a plain device copy and a plain read-only
// reduction, each streaming its bytes once with 16-byte non-temporal loads.
// The shapes are the fastest of a sweep on MI355X over unroll depth (4, 8,
// 16 loads in flight per thread), grid size (1024 to 16384 workgroups of 256
// threads) and access order: the read is fastest with each workgroup walking
// one contiguous chunk (16 loads in flight, 4096 workgroups), the copy with a
// grid-stride walk (4 loads in flight, 8192 workgroups).
#include "internal.hpp"

namespace sct {

constexpr int kCopyBlocks = 8192;
constexpr int kReadBlocks = 4096;
constexpr int kProbeThreads = 256;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// dst = src over n 16-byte words, grid-stride, 4 words in flight per thread.
__global__ __launch_bounds__(kProbeThreads) void k_stream_copy(const u32x4 *__restrict__ src,
                                                               u32x4 *__restrict__ dst, int64_t n)
{
    const int64_t stride = int64_t(gridDim.x) * kProbeThreads;
    int64_t i = int64_t(blockIdx.x) * kProbeThreads + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        u32x4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = __builtin_nontemporal_load(src + i + k * stride);
#pragma unroll
        for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(v[k], dst + i + k * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// One 32-bit xor-sum per workgroup of its contiguous chunk of src's n 16-byte
// words into part[block], 16 words in flight per thread (the result only
// keeps the loads from being removed).
__global__ __launch_bounds__(kProbeThreads) void k_stream_read(const u32x4 *__restrict__ src,
                                                               uint32_t *__restrict__ part, int64_t n)
{
    constexpr int U = 16;
    __shared__ uint32_t red[kProbeThreads];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = int64_t(blockIdx.x) * per, hi = lo + per < n ? lo + per : n;
    uint32_t acc = 0;
    int64_t i = lo + threadIdx.x;
    for (; i + (U - 1) * kProbeThreads < hi; i += U * kProbeThreads) {
        u32x4 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = __builtin_nontemporal_load(src + i + k * kProbeThreads);
#pragma unroll
        for (int k = 0; k < U; ++k) acc ^= v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
    }
    for (; i < hi; i += kProbeThreads) {
        const u32x4 v = __builtin_nontemporal_load(src + i);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kProbeThreads / 2; o >= 1; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] ^= red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace sct

using namespace sct;

extern "C" int radon_bandwidth_probe(int32_t mode, const void *src, void *dst, int64_t bytes,
                                     void *stream)
{
    clear_error();
    if (mode != RADON_PROBE_COPY && mode != RADON_PROBE_READ)
        return set_error(RADON_EINVAL, "mode must be RADON_PROBE_COPY or RADON_PROBE_READ (got %d)", mode);
    if (!src || !dst) return set_error(RADON_EINVAL, "src and dst must be non-NULL");
    if (bytes <= 0 || bytes % 16) return set_error(RADON_EINVAL, "bytes must be a positive multiple of 16");
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
        return set_error(RADON_EINVAL, "src and dst must be 16-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = bytes / 16;
    if (mode == RADON_PROBE_COPY) {
        k_stream_copy<<<kCopyBlocks, kProbeThreads, 0, s>>>(static_cast<const u32x4 *>(src),
                                                             static_cast<u32x4 *>(dst), n);
        return check_launch("k_stream_copy");
    }
    k_stream_read<<<kReadBlocks, kProbeThreads, 0, s>>>(static_cast<const u32x4 *>(src),
                                                         static_cast<uint32_t *>(dst), n);
    return check_launch("k_stream_read");
}
