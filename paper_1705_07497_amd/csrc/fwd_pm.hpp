// Forward product of a fused chunk from a pixel-major copy of its images.
//
// The per-image fused forward (fwd_quads) issues one gather per slot and
// image: a chunk of C images costs C load instructions per slot, each a
// scattered 8- or 16-byte read per lane, and the L1 processes every one.  Here
// the chunk is first copied to pixel-major order, xp[pixel][c] (a pixel's C
// values contiguous), so one 16-byte load fetches the pixel for VW = 4 FP32
// or 2 FP64 images and a slot needs 2 C / VW loads.  The copy costs one read
// and one or two writes of the chunk (the second, in transposed pixel order,
// serves the bundles of rays closer to horizontal).
//
// Lanes: the C / VW 16-byte groups of a pixel are split over GL adjacent
// lanes of one ray (each lane takes IQ = C / (VW GL) groups), so the 16-byte
// loads of GL neighbouring lanes are one contiguous run; the rest of the
// wave's 64 / BW lanes per ray take Q different runs of GL quads of the
// bundle.  Lane = (q, r, gl), gl fastest.
#pragma once

#include "products.hpp"

#include <type_traits>

namespace sct {

template <class TV, int C, int BW>
struct PmShape {
    static constexpr int VW = 16 / int(sizeof(TV));   // images per 16-byte load
    static constexpr int NG = C / VW;                 // 16-byte groups per pixel
    static constexpr int SUB = 64 / BW;               // lanes per ray in a wave
    static constexpr int GL = NG < SUB ? NG : SUB;    // lanes sharing a pixel's groups
    static constexpr int IQ = NG / GL;                // groups per lane
    static constexpr int Q = SUB / GL;                // quads per ray per wave step
    static_assert(C % VW == 0 && NG % GL == 0 && SUB % GL == 0, "pixel-major chunk shape");
};

// xp[(iy n + ix) C + c] = x[c][iy][ix] and, when xpT is given,
// xpT[(ix n + iy) C + c] = x[c][iy][ix], for the nb images of a chunk (the
// slots of images nb..C-1 are zero), through 16 x 16 pixel tiles in LDS.
template <class TV, int C>
__global__ __launch_bounds__(256) void k_pixel_major(const TV *__restrict__ x, TV *__restrict__ xp,
                                                     TV *__restrict__ xpT, int n, int64_t nn, int nb)
{
    __shared__ TV t[C][16][17];
    const int bx = blockIdx.x * 16, by = blockIdx.y * 16;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const bool in = by + ty < n && bx + tx < n;
    const int64_t at = int64_t(by + ty) * n + bx + tx;
#pragma unroll
    for (int c = 0; c < C; ++c) t[c][ty][tx] = (in && c < nb) ? x[int64_t(c) * nn + at] : TV(0);
    __syncthreads();
    // consecutive threads write consecutive elements: c fastest, then the
    // pixel along the output's row
    for (int e = threadIdx.x; e < 256 * C; e += 256) {
        const int c = e % C, p = e / C, px = p & 15, py = p >> 4;
        if (by + py < n && bx + px < n) xp[(int64_t(by + py) * n + bx + px) * C + c] = t[c][py][px];
    }
    if (xpT) {
        for (int e = threadIdx.x; e < 256 * C; e += 256) {
            const int c = e % C, p = e / C, py = p & 15, px = p >> 4;
            if (by + py < n && bx + px < n) xpT[(int64_t(bx + px) * n + by + py) * C + c] = t[c][py][px];
        }
    }
}

// Compile-time loop: f(std::integral_constant<int, J>) for J = J0 .. N-1.
template <int J, int N>
struct StaticFor {
    template <class F>
    __device__ __forceinline__ static void run(F &&f)
    {
        f(std::integral_constant<int, J>{});
        StaticFor<J + 1, N>::run(f);
    }
};
template <int N>
struct StaticFor<N, N> {
    template <class F>
    __device__ __forceinline__ static void run(F &&)
    {
    }
};

// v as held by lane J of this lane's group of GL adjacent lanes (GL = 1, 2
// or 4), through a DPP quad permutation of each 32-bit word (no LDS).
template <int GL, int J, class V>
__device__ __forceinline__ V group_bcast(const V &v)
{
    if constexpr (GL == 1) {
        return v;
    } else {
        static_assert(sizeof(V) % 4 == 0, "32-bit words");
        constexpr int perm = GL == 4 ? J * 0x55 : (J | (J << 2) | ((2 + J) << 4) | ((2 + J) << 6));
        constexpr int nw = int(sizeof(V) / 4);
        int w[nw];
        __builtin_memcpy(w, &v, sizeof(V));
#pragma unroll
        for (int k = 0; k < nw; ++k) w[k] = __builtin_amdgcn_mov_dpp(w[k], perm, 0xf, 0xf, false);
        V out;
        __builtin_memcpy(&out, w, sizeof(V));
        return out;
    }
}

// The quads [s0, s1) of one bundle for the C images of a pixel-major chunk
// (PAIR as in fwd_quads).  The GL lanes of a (q, r) group load GL
// consecutive quads of ray r with one set of stream loads and hand each
// quad's slots to the whole group, so every matrix entry is loaded once; a
// quad past s1 gets zero lengths (in-bounds gathers, no branch).  The group's
// lanes share ray r, so each derives the second lengths from its own ev.
template <class TM, class TV, int C, bool PAIR, bool COMPACT, int BW>
__device__ __forceinline__ void pm_quads(const FwdBundle &d, const u16x4 *__restrict__ I,
                                         const typename Quad<TM>::type *__restrict__ A,
                                         const typename Quad<TM>::type *__restrict__ Bv,
                                         const EdgeV<TV> &ev,
                                         const typename Vec16<TV>::type *__restrict__ xp, int n,
                                         int s0, int s1, int q, int r, int gl,
                                         TV (&acc)[PmShape<TV, C, BW>::IQ][PmShape<TV, C, BW>::VW])
{
    using S = PmShape<TV, C, BW>;
    using Qv = typename Quad<TM>::type;
    using V = typename Vec16<TV>::type;
    for (int tq = s0 + q * S::GL; tq < s1; tq += S::SUB) {
        const bool live = tq + gl < s1;
        const int e = (live ? tq + gl : tq) * BW + r;
        const u16x4 i4 = stream_load(I + e);
        Qv a4 = stream_load(A + e);
        a4 = live ? a4 : Qv(0);
        Qv b4;
        if constexpr (!COMPACT) {
            b4 = stream_load(Bv + e);
            b4 = live ? b4 : Qv(0);
        }
        StaticFor<0, S::GL>::run([&](auto jc) {
            constexpr int J = decltype(jc)::value;
            const u16x4 ij = group_bcast<S::GL, J>(i4);
            const Qv aj = group_bcast<S::GL, J>(a4);
            Qv bj;
            if constexpr (!COMPACT) bj = group_bcast<S::GL, J>(b4);
            const bool live_j = tq + J < s1;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int mu = d.m0 + 4 * (tq + J) + k;
                const int m = min(mu, n - 1);
                const int i0 = ij[k];
                const int ic = PAIR ? (i0 < n - 1 ? i0 : n - 2) : 0;
                const V *__restrict__ p = xp + (int64_t(m) * n + ic) * S::NG + gl;
                const TV a = TV(aj[k]);
                TV b;
                if constexpr (COMPACT) b = PAIR && live_j && i0 == ic ? second_len(ev, mu, a) : TV(0);
                else b = TV(bj[k]);
#pragma unroll
                for (int iq = 0; iq < S::IQ; ++iq) {
                    const V u = p[iq * S::GL];
                    if constexpr (PAIR) {
                        const V w = p[S::NG + iq * S::GL];
                        const V f = i0 == ic ? u : w;
#pragma unroll
                        for (int v = 0; v < S::VW; ++v) {
                            acc[iq][v] = fma(a, f[v], acc[iq][v]);
                            acc[iq][v] = fma(b, w[v], acc[iq][v]);
                        }
                    } else {
#pragma unroll
                        for (int v = 0; v < S::VW; ++v) acc[iq][v] = fma(a, u[v], acc[iq][v]);
                    }
                }
            }
        });
    }
}

// One bundle (quads [tq0, tq1), default all) for the nbc images of a
// pixel-major chunk xp (the gather class of the bundle): y[c * ystride +
// ray] for c < nbc.  Sums over q with shuffles and over the W waves in LDS,
// in a fixed order.
template <class TM, class TV, int W, int C, int BW>
__device__ __forceinline__ void pm_bundle(const FwdBundle &d, const uint16_t *__restrict__ idx,
                                          const TM *__restrict__ v0, const TM *__restrict__ v1,
                                          const RayEdge *__restrict__ edge,
                                          const TV *__restrict__ xp, TV *__restrict__ y, int n,
                                          int64_t ystride, int nbc, int tq0 = 0, int tq1 = -1)
{
    using S = PmShape<TV, C, BW>;
    using Qv = typename Quad<TM>::type;
    using V = typename Vec16<TV>::type;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int gl = lane % S::GL, r = (lane / S::GL) % BW, q = lane / (S::GL * BW);
    const int nq = tq1 < 0 ? (d.nrows >> 2) - tq0 : tq1 - tq0;
    const int s0 = tq0 + (nq * wave) / W, s1 = tq0 + (nq * (wave + 1)) / W;
    const u16x4 *__restrict__ I = reinterpret_cast<const u16x4 *>(idx + d.off);
    const Qv *__restrict__ A = reinterpret_cast<const Qv *>(v0 + d.off);
    const int64_t ray = bundle_ray(d, r);
    const V *__restrict__ xv = reinterpret_cast<const V *>(xp);
    TV acc[S::IQ][S::VW];
#pragma unroll
    for (int iq = 0; iq < S::IQ; ++iq)
#pragma unroll
        for (int v = 0; v < S::VW; ++v) acc[iq][v] = TV(0);
    if (v1) {   // both lengths stored
        const Qv *__restrict__ Bv = reinterpret_cast<const Qv *>(v1 + d.off);
        const EdgeV<TV> ev{};
        if (n >= 2)
            pm_quads<TM, TV, C, true, false, BW>(d, I, A, Bv, ev, xv, n, s0, s1, q, r, gl, acc);
        else
            pm_quads<TM, TV, C, false, false, BW>(d, I, A, Bv, ev, xv, n, s0, s1, q, r, gl, acc);
    } else {    // compact: second lengths from the ray's chord
        const EdgeV<TV> ev = load_edge<TV>(edge, ray);
        if (n >= 2)
            pm_quads<TM, TV, C, true, true, BW>(d, I, A, nullptr, ev, xv, n, s0, s1, q, r, gl, acc);
        else
            pm_quads<TM, TV, C, false, true, BW>(d, I, A, nullptr, ev, xv, n, s0, s1, q, r, gl, acc);
    }
#pragma unroll
    for (int iq = 0; iq < S::IQ; ++iq)
#pragma unroll
        for (int v = 0; v < S::VW; ++v)
#pragma unroll
            for (int o = S::GL * BW; o < 64; o <<= 1) acc[iq][v] += __shfl_xor(acc[iq][v], o);
    if constexpr (W > 1) {
        __shared__ TV red[W][C][BW];
        if (q == 0) {
#pragma unroll
            for (int iq = 0; iq < S::IQ; ++iq)
#pragma unroll
                for (int v = 0; v < S::VW; ++v) red[wave][(iq * S::GL + gl) * S::VW + v][r] = acc[iq][v];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int iq = 0; iq < S::IQ; ++iq)
#pragma unroll
                for (int v = 0; v < S::VW; ++v) {
                    const int c = (iq * S::GL + gl) * S::VW + v;
                    acc[iq][v] = red[0][c][r];
#pragma unroll
                    for (int w = 1; w < W; ++w) acc[iq][v] += red[w][c][r];
                }
        }
        __syncthreads();   // red is reused by the next bundle
    }
    if (wave == 0 && q == 0 && ray >= 0) {
#pragma unroll
        for (int iq = 0; iq < S::IQ; ++iq)
#pragma unroll
            for (int v = 0; v < S::VW; ++v) {
                const int c = (iq * S::GL + gl) * S::VW + v;
                if (c < nbc) y[int64_t(c) * ystride + ray] = acc[iq][v];
            }
    }
}

// Forward of one pixel-major chunk over the operator's bundles (as k_fwd).
template <class TM, class TV, int W, int C, int BW>
__global__ __launch_bounds__(64 * W) void k_fwd_pm(const FwdBundle *__restrict__ fb,
                                                   const int32_t *__restrict__ order, int64_t n_order,
                                                   const uint16_t *__restrict__ idx,
                                                   const TM *__restrict__ v0, const TM *__restrict__ v1,
                                                   const RayEdge *__restrict__ edge,
                                                   const TV *__restrict__ xp, const TV *__restrict__ xpT,
                                                   TV *__restrict__ y, int n, int64_t rows, int nbc)
{
    for (int64_t o = blockIdx.x; o < n_order; o += gridDim.x) {
        const int B = order[o];
        if (B < 0) continue;           // padding entry (uniform per block)
        const FwdBundle d = fb[B];
        pm_bundle<TM, TV, W, C, BW>(d, idx, v0, v1, edge, d.horiz ? xpT : xp, y, n, rows, nbc);
    }
}

// Line-banded forward of one pixel-major chunk (as k_fwd_band): partials
// part[image][band][ray].  The items are handed out in list order through
// one ticket counter per XCD (entry o belongs to XCD o % 8, block i runs on
// XCD i % 8): with a static round-robin the blocks of an XCD drift apart
// over the items and work on several bands at once.
template <class TM, class TV, int W, int C, int BW>
__global__ __launch_bounds__(64 * W) void k_fwd_pm_band(const FwdBundle *__restrict__ fb,
                                                        const int2 *__restrict__ order, int64_t n_order,
                                                        const uint16_t *__restrict__ idx,
                                                        const TM *__restrict__ v0,
                                                        const TM *__restrict__ v1,
                                                        const RayEdge *__restrict__ edge,
                                                        const TV *__restrict__ xp,
                                                        const TV *__restrict__ xpT, TV *__restrict__ part,
                                                        int n, int64_t rows, int n_bands, int lines,
                                                        int nbc, uint32_t *__restrict__ tickets)
{
    const int64_t stride = int64_t(n_bands) * rows;   // one image's partials
    __shared__ int64_t next;
    const int xcd = int(blockIdx.x & 7u);
    uint32_t *const counter = tickets + xcd * kTicketStride;
    for (;;) {
        if (threadIdx.x == 0) next = 8 * int64_t(atomicAdd(counter, 1u)) + xcd;
        __syncthreads();
        const int64_t o = next;
        __syncthreads();   // next is written again only after every wave has read it
        if (o >= n_order) break;
        const int2 it = order[o];
        if (it.x < 0) continue;        // padding entry (uniform per block)
        const FwdBundle d = fb[it.x];
        const int nq = d.nrows >> 2;
        const int lo = it.y * lines - d.m0, hi = lo + lines;
        const int tq0 = lo <= 0 ? 0 : min(nq, (lo + 3) >> 2);
        const int tq1 = hi <= 0 ? 0 : min(nq, (hi + 3) >> 2);
        pm_bundle<TM, TV, W, C, BW>(d, idx, v0, v1, edge, d.horiz ? xpT : xp, part + int64_t(it.y) * rows, n,
                                    stride, nbc, tq0, tq1);
    }
}

}  // namespace sct
