// CG state and the vector helpers shared by the single-operator solvers
// (solve.hip) and the multi-operator CG (multi.hip).
#pragma once

#include "internal.hpp"

namespace sct {

// Per right-hand side CG state at the start of an iteration, in a two-slot
// ring indexed by iteration parity: every kernel reads slot it%2 and only a
// later kernel writes slot (it+1)%2, so no kernel reads what it writes.
struct CgState {
    double rho, rho0;
    int32_t stopped, iters, breakdown, pad;
};

// Result of the step-length decision of one iteration (also a 2-slot ring).
struct CgStep {
    double a, gamma;
    int32_t stopped, pad;
};

// Step decision of one CG iteration: stop on rho == 0, on the relative
// tolerance (rtol > 0), or on a breakdown (gamma <= 0 or non-finite: returns
// 2); otherwise *a = rho / gamma and 0.
__device__ inline int cg_decide(const CgState &c, double gamma, double rtol, double *a)
{
    *a = 0.0;
    if (c.stopped) return c.stopped;
    if (c.rho == 0.0 || (rtol > 0.0 && sqrt(c.rho) <= rtol * sqrt(c.rho0))) return 1;
    if (!(gamma > 0.0) || !isfinite(gamma)) return 2;
    *a = c.rho / gamma;
    return 0;
}

constexpr int kVecThreads = 256;

inline int vec_blocks(int64_t nn)
{
    const int64_t b = (nn + 4 * kVecThreads - 1) / (4 * kVecThreads);
    return int(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

inline int tiles_of(int n) { return (n + 31) / 32; }

__device__ inline double block_sum(double v, double *red)
{
    // fixed order over the block (blockDim.x * blockDim.y threads, a multiple
    // of 64): a butterfly inside each wave (every lane ends with the same
    // bits, as IEEE addition commutes), then the wave sums in wave order
    const int nt = blockDim.x * blockDim.y;
    const int t = threadIdx.y * blockDim.x + threadIdx.x;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < (nt >> 6); ++w) r += red[w];
    __syncthreads();
    return r;
}

__device__ inline double sum_part_block(const double *__restrict__ part, int64_t count, double *red)
{
    // each thread adds its strided share in index order; the loads of a group
    // of kG are issued before the first add, so one memory latency covers the
    // group instead of one per element (the sum is the same either way)
    constexpr int kG = 8;
    const int64_t st = blockDim.x;
    double v = 0.0;
    int64_t i = threadIdx.x;
    for (; i + (kG - 1) * st < count; i += kG * st) {
        double t[kG];
#pragma unroll
        for (int k = 0; k < kG; ++k) t[k] = part[i + k * st];
#pragma unroll
        for (int k = 0; k < kG; ++k) v += t[k];
    }
    for (; i < count; i += st) v += part[i];
    return block_sum(v, red);
}

template <class T>
__global__ __launch_bounds__(kVecThreads) void k_fill(T *__restrict__ x, T v, int64_t count)
{
    for (int64_t i = int64_t(blockIdx.x) * kVecThreads + threadIdx.x; i < count;
         i += int64_t(gridDim.x) * kVecThreads)
        x[i] = v;
}

template <class T>
__global__ __launch_bounds__(kVecThreads) void k_copy(const T *__restrict__ a, T *__restrict__ r,
                                                       int64_t count)
{
    for (int64_t i = int64_t(blockIdx.x) * kVecThreads + threadIdx.x; i < count;
         i += int64_t(gridDim.x) * kVecThreads)
        r[i] = a[i];
}

}  // namespace sct
