// Forward product of an operator stored by the symmetries of the square
// (Op::sym).  Its bundles hold only the rays of the measured angles theta in
// [0, pi/4] (rays closer to vertical: slots along image rows).  Each such ray
// stands for up to three more measured rays with the same bin, its images
// under maps of the pixel grid onto itself:
//   pi - theta    x -> -x:        row m, pixels (n-2-q, n-1-q), lengths swapped;
//   pi/2 - theta  the transpose:  line m of the transposed image, pixels (q, q+1);
//   pi/2 + theta  both:           line n-1-m of the transposed image, (q, q+1),
// where (q, q+1) are the pixels of the stored slot on row m (a ray through
// pixel (ix, iy) at theta passes through (n-1-ix, iy), (iy, ix) and
// (n-1-iy, ix) at the three other angles, at the same distance from the
// centre, so with the same lengths).  partner[a] gives the three measured
// angles for stored angle a (-1: not measured, or the angle itself or
// another partner).  One slot load serves up to four gathers.
#pragma once

#include "products.hpp"

namespace sct {

template <class TM, class TV, bool COMPACT, int BW>
__device__ __forceinline__ void sym_quads(const FwdBundle &d, const u16x4 *__restrict__ I,
                                          const typename Quad<TM>::type *__restrict__ A,
                                          const typename Quad<TM>::type *__restrict__ Bv,
                                          const EdgeV<TV> &ev, const TV *__restrict__ x,
                                          const TV *__restrict__ xT, int n, int s0, int s1, int q, int r,
                                          TV (&acc)[4])
{
    using Q = typename Quad<TM>::type;
    using P = typename PairU<TV>::type;
    constexpr int G = 64 / BW;
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
            const bool inb = i0 < n - 1;           // the slot has a second pixel
            const int ic = inb ? i0 : n - 2;       // its pair, kept inside the line
            const int fc = inb ? n - 2 - i0 : 0;   // the mirrored pair
            const TV a = TV(a4[k]);
            TV b;
            if constexpr (COMPACT) b = inb ? second_len(ev, mu, a) : TV(0);
            else b = TV(b4[k]);
            const P p0 = *reinterpret_cast<const P *>(x + int64_t(m) * n + ic);
            const P p1 = *reinterpret_cast<const P *>(x + int64_t(m) * n + fc);
            const P p2 = *reinterpret_cast<const P *>(xT + int64_t(m) * n + ic);
            const P p3 = *reinterpret_cast<const P *>(xT + int64_t(n - 1 - m) * n + ic);
            acc[0] = fma(a, inb ? p0.x : p0.y, acc[0]);
            acc[0] = fma(b, p0.y, acc[0]);
            acc[1] = fma(a, inb ? p1.y : p1.x, acc[1]);
            acc[1] = fma(b, p1.x, acc[1]);
            acc[2] = fma(a, inb ? p2.x : p2.y, acc[2]);
            acc[2] = fma(b, p2.y, acc[2]);
            acc[3] = fma(a, inb ? p3.x : p3.y, acc[3]);
            acc[3] = fma(b, p3.y, acc[3]);
        }
    }
}

// One image per blockIdx.y; persistent loop over the stored bundles as k_fwd.
template <class TM, class TV, int W, int BW>
__global__ __launch_bounds__(64 * W) void k_fwd_sym(const FwdBundle *__restrict__ fb,
                                                    const int32_t *__restrict__ order, int64_t n_order,
                                                    const uint16_t *__restrict__ idx,
                                                    const TM *__restrict__ v0, const TM *__restrict__ v1,
                                                    const RayEdge *__restrict__ edge,
                                                    const int4 *__restrict__ partner,
                                                    const TV *__restrict__ x, const TV *__restrict__ xT,
                                                    TV *__restrict__ y, int n, int nb, int64_t nn, int64_t rows)
{
    using Q = typename Quad<TM>::type;
    const int64_t img = blockIdx.y;
    const TV *__restrict__ xb = x + img * nn;
    const TV *__restrict__ xTb = xT + img * nn;
    TV *__restrict__ yb = y + img * rows;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int r = lane % BW, q = lane / BW;
    __shared__ TV red[W > 1 ? W : 1][4][BW];
    for (int64_t o = blockIdx.x; o < n_order; o += gridDim.x) {
        const int B = order[o];
        if (B < 0) continue;   // padding entry (uniform per block)
        const FwdBundle d = fb[B];
        const int nq = d.nrows >> 2;
        const int s0 = (nq * wave) / W, s1 = (nq * (wave + 1)) / W;
        const u16x4 *__restrict__ I = reinterpret_cast<const u16x4 *>(idx + d.off);
        const Q *__restrict__ A = reinterpret_cast<const Q *>(v0 + d.off);
        const int64_t ray = bundle_ray(d, r);
        TV acc[4] = {TV(0), TV(0), TV(0), TV(0)};
        if (v1) {
            const Q *__restrict__ Bv = reinterpret_cast<const Q *>(v1 + d.off);
            const EdgeV<TV> ev{};
            sym_quads<TM, TV, false, BW>(d, I, A, Bv, ev, xb, xTb, n, s0, s1, q, r, acc);
        } else {
            const EdgeV<TV> ev = load_edge<TV>(edge, ray);
            sym_quads<TM, TV, true, BW>(d, I, A, nullptr, ev, xb, xTb, n, s0, s1, q, r, acc);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int o2 = BW; o2 < 64; o2 <<= 1) acc[j] += __shfl_xor(acc[j], o2);
        }
        if constexpr (W > 1) {
            if (q == 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j) red[wave][j][r] = acc[j];
            }
            __syncthreads();
            if (wave == 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[j] = red[0][j][r];
#pragma unroll
                    for (int w = 1; w < W; ++w) acc[j] += red[w][j][r];
                }
            }
            __syncthreads();   // red is reused by the next bundle
        }
        if (wave == 0 && q == 0 && ray >= 0) {
            const int a = int(ray / nb), bin = int(ray % nb);
            const int4 pa = partner[a];
            yb[ray] = acc[0];
            if (pa.x >= 0) yb[int64_t(pa.x) * nb + bin] = acc[1];
            if (pa.y >= 0) yb[int64_t(pa.y) * nb + bin] = acc[2];
            if (pa.z >= 0) yb[int64_t(pa.z) * nb + bin] = acc[3];
        }
    }
}

template <class TM, class TV, int W, int BW>
inline void fwd_sym_w(const Op &op, const TV *x, const TV *xT, TV *y, int batch, hipStream_t s)
{
    const int64_t g = op.n_order < kPersistentBlocks ? op.n_order : kPersistentBlocks;
    k_fwd_sym<TM, TV, W, BW><<<dim3(unsigned(g), unsigned(batch)), 64 * W, 0, s>>>(
        op.fb, op.fb_order, op.n_order, op.f_idx, static_cast<const TM *>(op.f_v0),
        static_cast<const TM *>(op.f_v1), op.f_edge, op.f_partner, x, xT, y, op.n, op.n_bins, op.nn, op.rows);
}

// Forward of a symmetric operator: needs the transposed images.
template <class TM, class TV, int BW>
inline int launch_fwd_sym(const Op &op, const TV *x, const TV *xT, TV *y, int batch, hipStream_t s)
{
    if (!xT) return set_error(RADON_EINVAL, "a symmetric operator's forward needs the transposed images");
    if (op.tune.fwd_waves == 2) fwd_sym_w<TM, TV, 2, BW>(op, x, xT, y, batch, s);
    else fwd_sym_w<TM, TV, 4, BW>(op, x, xT, y, batch, s);
    return check_launch("k_fwd_sym");
}

}  // namespace sct
