// Device-side bodies of the sparse products, shared by the single-operator
// kernels (apply.hip) and the multi-operator kernels (multi.hip).
#pragma once

#include "internal.hpp"

namespace sct {

// xT[b][ix][iy] = x[b][iy][ix] through a padded 32x32 LDS tile.
template <class T>
__global__ __launch_bounds__(256) void k_transpose(const T *__restrict__ x, T *__restrict__ xT,
                                                   int n, int64_t nn)
{
    __shared__ T tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int64_t boff = int64_t(blockIdx.z) * nn;
    for (int i = threadIdx.y; i < 32; i += 8) {
        const int iy = by + i, ix = bx + threadIdx.x;
        if (iy < n && ix < n) tile[i][threadIdx.x] = x[boff + int64_t(iy) * n + ix];
    }
    __syncthreads();
    for (int i = threadIdx.y; i < 32; i += 8) {
        const int ix = bx + i, iy = by + threadIdx.x;
        if (ix < n && iy < n) xT[boff + int64_t(ix) * n + iy] = tile[threadIdx.x][i];
    }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
template <class T> struct Quad;
template <> struct Quad<float> { using type = f32x4; };
template <> struct Quad<double> { using type = f64x4; };

// Two adjacent vector elements fetched with one 16-byte load (8-byte aligned).
typedef double f64x2u __attribute__((ext_vector_type(2), aligned(8)));
typedef float f32x2u __attribute__((ext_vector_type(2), aligned(4)));
template <class T> struct PairU;
template <> struct PairU<float> { using type = f32x2u; };
template <> struct PairU<double> { using type = f64x2u; };

// 16 bytes of vector elements (4 FP32 or 2 FP64), 16-byte aligned.
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <class TV> struct Vec16;
template <> struct Vec16<float> { using type = f32x4; };
template <> struct Vec16<double> { using type = f64x2; };

// The matrix streams are read exactly once per product: non-temporal loads
// keep them from evicting the gathered vector from the caches.
template <class V>
__device__ inline V stream_load(const V *p)
{
    return __builtin_nontemporal_load(p);
}

// A lane's ray, for the second lengths of its slots (RayEdge in the vector
// type; a lane without a ray gets mf > ml, so every second length is 0).
template <class TV>
struct EdgeV {
    TV chord, w1f, w1l;
    int mf, ml;
};

template <class TV>
__device__ __forceinline__ EdgeV<TV> load_edge(const RayEdge *__restrict__ edge, int64_t ray)
{
    EdgeV<TV> v;
    v.chord = v.w1f = v.w1l = TV(0);
    v.mf = 1;
    v.ml = 0;
    if (ray >= 0) {
        const RayEdge e = edge[ray];
        v.chord = TV(e.chord);
        v.w1f = TV(e.w1f);
        v.w1l = TV(e.w1l);
        v.mf = e.mf;
        v.ml = e.ml;
    }
    return v;
}

// Length in the second pixel of the slot on major line mu (unclamped) whose
// first length is w0: the chord minus w0 on the lines the ray crosses from
// side to side, the stored value on its first and last lines, 0 outside.
template <class TV>
__device__ __forceinline__ TV second_len(const EdgeV<TV> &e, int mu, TV w0)
{
    TV w = e.chord - w0;
    w = mu == e.mf ? e.w1f : w;
    w = mu == e.ml ? e.w1l : w;
    return (mu < e.mf || mu > e.ml) ? TV(0) : w;
}

// One workgroup of W waves per ray bundle (block -> bundle through `order`,
// which places bundles of rays closer to vertical and closer to horizontal on
// different XCDs, so each XCD's L2 caches only x or only its transpose).
// Lane = (quad offset q in 0..64/BW-1, ray r in 0..BW-1): a lane reads a quad
// (4 consecutive major lines of its ray) with 16-byte loads, the 64 lanes of
// a wave read 64 consecutive quads, and the BW lanes of one q gather from the
// same image line at neighbouring positions.  Wave w covers its share of the
// bundle's quads; partial sums are combined over q with shuffles and over the
// waves in LDS, in a fixed order.
// Several right-hand sides: blockIdx.y selects a chunk of up to BC images that
// share every matrix load (the fused multi-RHS product), one accumulator each.
// The quads of wave shares [s0, s1) of one bundle for up to BC images.
// PAIR (n >= 2): one 16-byte load fetches both pixels of a slot; a slot at
// the last column has no second pixel (its second length is 0), so its pair
// starts at n-2.
// The test is a template parameter so that the loop body has no branch: a
// branch around each gather makes every gather wait for all loads in flight.
template <class TM, class TV, int BC, bool PAIR, bool COMPACT, int BW>
__device__ __forceinline__ void fwd_quads(const FwdBundle &d, const u16x4 *__restrict__ I,
                                          const typename Quad<TM>::type *__restrict__ A,
                                          const typename Quad<TM>::type *__restrict__ Bv,
                                          const EdgeV<TV> &ev, const TV *__restrict__ img, int n,
                                          int64_t nn, int nbc, int s0, int s1, int q, int r, TV *acc)
{
    using Q = typename Quad<TM>::type;
    using P = typename PairU<TV>::type;
    constexpr int G = 64 / BW;   // quads a wave covers per step
#pragma unroll 2
    for (int tq = s0 + q; tq < s1; tq += G) {
        const int e = tq * BW + r;
        const u16x4 i4 = stream_load(I + e);
        const Q a4 = stream_load(A + e);
        Q b4;
        if constexpr (!COMPACT) b4 = stream_load(Bv + e);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int mu = d.m0 + 4 * tq + k;
            const int m = min(mu, n - 1);
            const int i0 = i4[k];
            const int ic = PAIR ? (i0 < n - 1 ? i0 : n - 2) : 0;
            const int64_t at = int64_t(m) * n + ic;
            const TV a = TV(a4[k]);
            TV b;
            if constexpr (COMPACT) b = PAIR && i0 == ic ? second_len(ev, mu, a) : TV(0);
            else b = TV(b4[k]);
#pragma unroll
            for (int c = 0; c < BC; ++c) {
                if (BC == 1 || c < nbc) {
                    const TV *__restrict__ line = img + int64_t(c) * nn;
                    if constexpr (PAIR) {
                        const P pr = *reinterpret_cast<const P *>(line + at);
                        acc[c] = fma(a, i0 == ic ? pr.x : pr.y, acc[c]);
                        acc[c] = fma(b, pr.y, acc[c]);
                    } else {
                        acc[c] = fma(a, line[0], acc[c]);
                    }
                }
            }
        }
    }
}

// fwd_bundle does one bundle for up to BC images (img and y point at the
// first image of the chunk, nbc of them present); k_fwd loops over the
// bundles of one operator, k_multi_fwd over those of several.
// [tq0, tq1) restricts the bundle to a range of its quads (the line-banded
// forward); the default is the whole bundle.
template <class TM, class TV, int W, int BC, int BW>
__device__ __forceinline__ void fwd_bundle(const FwdBundle &d, const uint16_t *__restrict__ idx,
                                           const TM *__restrict__ v0, const TM *__restrict__ v1,
                                           const RayEdge *__restrict__ edge,
                                           const TV *__restrict__ img, TV *__restrict__ y, int n,
                                           int64_t nn, int64_t rows, int nbc, int tq0 = 0,
                                           int tq1 = -1)
{
    using Q = typename Quad<TM>::type;
    static_assert(BW == 16 || BW == 32 || BW == 64, "bundle width");
    // the wave index is uniform: readfirstlane lets the compiler see that
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int r = lane % BW, q = lane / BW;
    const int nq = tq1 < 0 ? (d.nrows >> 2) - tq0 : tq1 - tq0;
    const int s0 = tq0 + (nq * wave) / W, s1 = tq0 + (nq * (wave + 1)) / W;
    const u16x4 *__restrict__ I = reinterpret_cast<const u16x4 *>(idx + d.off);
    const Q *__restrict__ A = reinterpret_cast<const Q *>(v0 + d.off);
    const int64_t ray = bundle_ray(d, r);
    TV acc[BC];
#pragma unroll
    for (int c = 0; c < BC; ++c) acc[c] = TV(0);
    if (v1) {   // both lengths stored
        const Q *__restrict__ Bv = reinterpret_cast<const Q *>(v1 + d.off);
        const EdgeV<TV> ev{};
        if (n >= 2)
            fwd_quads<TM, TV, BC, true, false, BW>(d, I, A, Bv, ev, img, n, nn, nbc, s0, s1, q, r, acc);
        else
            fwd_quads<TM, TV, BC, false, false, BW>(d, I, A, Bv, ev, img, n, nn, nbc, s0, s1, q, r, acc);
    } else {    // compact: second lengths from the ray's chord
        const EdgeV<TV> ev = load_edge<TV>(edge, ray);
        if (n >= 2)
            fwd_quads<TM, TV, BC, true, true, BW>(d, I, A, nullptr, ev, img, n, nn, nbc, s0, s1, q, r, acc);
        else
            fwd_quads<TM, TV, BC, false, true, BW>(d, I, A, nullptr, ev, img, n, nn, nbc, s0, s1, q, r, acc);
    }
#pragma unroll
    for (int c = 0; c < BC; ++c) {
#pragma unroll
        for (int o = BW; o < 64; o <<= 1) acc[c] += __shfl_xor(acc[c], o);
    }
    if constexpr (W > 1) {
        __shared__ TV red[W][BC][BW];
        if (q == 0) {
#pragma unroll
            for (int c = 0; c < BC; ++c) red[wave][c][r] = acc[c];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int c = 0; c < BC; ++c) {
                acc[c] = red[0][c][r];
#pragma unroll
                for (int w = 1; w < W; ++w) acc[c] += red[w][c][r];
            }
        }
        __syncthreads();   // red is reused by the next bundle
    }
    if (wave == 0 && q == 0 && ray >= 0) {
#pragma unroll
        for (int c = 0; c < BC; ++c)
            if (c < nbc) y[int64_t(c) * rows + ray] = acc[c];
    }
}

// y[ray] = sum of the ray's band partials, in band order (the bands its
// bundle's quads start in; none for a bundle that misses the image).
template <class TV>
__global__ __launch_bounds__(256) void k_fwd_band_sum(const FwdBundle *__restrict__ fb,
                                                      const TV *__restrict__ part, TV *__restrict__ y,
                                                      int64_t rows, int nb, BundleMap bm,
                                                      int n_bands, int lines)
{
    const int64_t ray = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ray >= rows) return;
    const int b = blockIdx.y;
    const int a = int(ray / nb), bin = int(ray % nb);
    int lane = 0;
    const FwdBundle d = fb[bm.bundle_of(a, bin, &lane)];
    TV acc = TV(0);
    if (d.nrows > 0) {
        const int lo = d.m0 / lines, hi = (d.m0 + d.nrows - 4) / lines;
        const TV *p = part + int64_t(b) * n_bands * rows + ray;
        // groups of four loads in flight, added in band order
        int band = lo;
        for (; band + 3 <= hi; band += 4) {
            TV t[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) t[k] = p[int64_t(band + k) * rows];
#pragma unroll
            for (int k = 0; k < 4; ++k) acc += t[k];
        }
        for (; band <= hi; ++band) acc += p[int64_t(band) * rows];
    }
    y[int64_t(b) * rows + ray] = acc;
}

// Clears the 8 ticket counters (kTicketStride apart) before each launch that
// uses them: a kernel, not a memset node, so the sequence can be captured in
// a graph.
__global__ inline void k_ticket_reset(uint32_t *__restrict__ tickets)
{
    if (threadIdx.x < 8) tickets[threadIdx.x * kTicketStride] = 0u;
}

// (K^T K x)_j, the Neumann 5-point Laplacian.  The four neighbours load
// unconditionally, so their latencies overlap: a neighbour missing at the
// image edge reads x_j itself, whose difference is exactly zero.
template <class T>
__device__ inline T ktk_at(const T *__restrict__ xb, int64_t j, int n, T xj)
{
    const int iy = int(j / n), ix = int(j % n);
    const T l = xb[ix > 0 ? j - 1 : j], r = xb[ix < n - 1 ? j + 1 : j];
    const T d = xb[iy > 0 ? j - n : j], u = xb[iy < n - 1 ? j + n : j];
    T k = T(0);
    k += xj - l;
    k += xj - r;
    k += xj - d;
    k += xj - u;
    return k;
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Quads of one tile whose base bins a wave stages in LDS at a time: one
// 2-byte load per lane.  With the bases in LDS the band address of a quad
// waits only on LDS, so the quad's matrix streams are not held back behind a
// global load of its base.
constexpr int kBaseChunk = kAdjLanes / 4;

// Single right-hand side adjoint sum for 8x8 tile g (the layout and the band
// staging are described at k_adj below): returns the tile's 64 sums in the
// lanes of wave 0 (other waves return their own share).  `band` is this
// block's [W][4][kAdjBand] LDS staging area, `bases` its [W][kAdjLanes] one.
template <class TM, class T, int W>
__device__ __forceinline__ T adj_tile1(int64_t g, const uint32_t *__restrict__ Rl,
                                       const uint16_t *__restrict__ base,
                                       const typename Quad<TM>::type *__restrict__ A,
                                       const typename Quad<TM>::type *__restrict__ Bv, int n_meas,
                                       int n_aq, int nb, const T *__restrict__ yb, T *band,
                                       uint16_t *bases)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int q0 = (n_aq * wave) / W, q1 = (n_aq * (wave + 1)) / W;
    const int kk = lane >> 4, ee = lane & 15;   // this lane's band element
    T *__restrict__ my = band + wave * 4 * kAdjBand;
    uint16_t *__restrict__ mb = bases + wave * kAdjLanes;
    T acc = T(0);
    for (int c0 = q0; c0 < q1; c0 += kBaseChunk) {
        const int nc = min(kBaseChunk, q1 - c0);
        if (lane < 4 * nc) mb[lane] = base[(g * n_aq + c0) * 4 + lane];
        __builtin_amdgcn_wave_barrier();
#pragma unroll 2
        for (int j = 0; j < nc; ++j) {
            const int aq = c0 + j;
            const int64_t gq = g * n_aq + aq;
            const int a_band = min(4 * aq + kk, n_meas - 1);
            const int b_band = min(int(mb[4 * j + kk]) + ee, nb - 1);
            const T yv = yb[int64_t(a_band) * nb + b_band];
            const int64_t e = gq * kAdjLanes + lane;
            const uint32_t r4 = stream_load(Rl + e);
            const auto a4 = stream_load(A + e);
            const auto c4 = stream_load(Bv + e);
            my[lane] = yv;
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int rb = int((r4 >> (8 * k)) & 0xffu);
                acc = fma(T(a4[k]), my[k * kAdjBand + rb], acc);
                acc = fma(T(c4[k]), my[k * kAdjBand + rb + 1], acc);
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    if constexpr (W > 1) {
        __shared__ T red[W][64];
        red[wave][lane] = acc;
        __syncthreads();
        if (wave == 0) {
            acc = red[0][lane];
#pragma unroll
            for (int w = 1; w < W; ++w) acc += red[w][lane];
        }
        __syncthreads();   // red is reused by the next tile
    }
    return acc;
}

// Epilogue of tile g for wave 0's lane: out = alpha*acc + lambda*(K^T K x) +
// sigma*x; returns x_j * out_j (0 outside the image or without x).
template <class T>
__device__ __forceinline__ double adj_epilogue(int64_t g, int lane, T acc, const T *__restrict__ xb,
                                               T *__restrict__ ob, T alpha, T lambda, T sigma,
                                               int n, int tiles)
{
    const int iy = int(g / tiles) * 8 + (lane >> 3), ix = int(g % tiles) * 8 + (lane & 7);
    if (iy >= n || ix >= n) return 0.0;
    const int64_t j = int64_t(iy) * n + ix;
    T o = alpha * acc;
    double d = 0.0;
    if (xb) {
        const T xj = xb[j];
        if (lambda != T(0)) o += lambda * ktk_at(xb, j, n, xj);
        if (sigma != T(0)) o += sigma * xj;
        d = double(xj) * double(o);
    }
    ob[j] = o;
    return d;
}

}  // namespace sct
