// Forward-product kernels and their launchers for one bundle width.  Each
// width is compiled in a translation unit of its own (fwd16.hip, fwd32.hip,
// fwd64.hip) that instantiates launch_fwd_bw for the three operator kinds;
// apply.hip's launch_fwd picks the operator's width.
#pragma once

#include "fwd_pm.hpp"
#include "fwd_sym.hpp"

namespace sct {

// Forward product of one operator: persistent loop over its ray bundles
// (see fwd_bundle).
template <class TM, class TV, int W, int BC, int BW>
__global__ __launch_bounds__(64 * W) void k_fwd(const FwdBundle *__restrict__ fb,
                                                const int32_t *__restrict__ order, int64_t n_order,
                                                const uint16_t *__restrict__ idx,
                                                const TM *__restrict__ v0, const TM *__restrict__ v1,
                                                const RayEdge *__restrict__ edge,
                                                const TV *__restrict__ x, const TV *__restrict__ xT,
                                                TV *__restrict__ y, int n, int64_t nn, int64_t rows,
                                                int batch)
{
    const int b0 = int(blockIdx.y) * BC;
    const int nbc = min(BC, batch - b0);
    // persistent: the grid is a multiple of 8 blocks, so block i stays on XCD
    // i % 8 and order[] keeps one gather class per XCD
    for (int64_t o = blockIdx.x; o < n_order; o += gridDim.x) {
        const int B = order[o];
        if (B < 0) continue;           // padding entry (uniform per block)
        const FwdBundle d = fb[B];
        fwd_bundle<TM, TV, W, BC, BW>(d, idx, v0, v1, edge, (d.horiz ? xT : x) + int64_t(b0) * nn,
                                      y + int64_t(b0) * rows, n, nn, rows, nbc);
    }
}

// Line-banded forward: work item (bundle, band) covers the bundle's quads
// whose first line lies in lines [band L, (band + 1) L).  Items are ordered
// band-major on each XCD, so the blocks of an XCD gather from one band of
// the image (or its transpose) at a time and keep it in that XCD's L2 across
// all angles.  The items are handed out in list order through one ticket
// counter per XCD (entry o belongs to XCD o % 8, block i runs on XCD i % 8):
// with a static round-robin the blocks of an XCD drift apart over the items
// and work on several bands at once.  Each item writes its partial sums to
// part[image][band][ray].  A chunk of up to BC images shares every matrix
// load, as in k_fwd.
template <class TM, class TV, int W, int BC, int BW>
__global__ __launch_bounds__(64 * W) void k_fwd_band(const FwdBundle *__restrict__ fb,
                                                     const int2 *__restrict__ order, int64_t n_order,
                                                     const uint16_t *__restrict__ idx,
                                                     const TM *__restrict__ v0, const TM *__restrict__ v1,
                                                const RayEdge *__restrict__ edge,
                                                     const TV *__restrict__ x, const TV *__restrict__ xT,
                                                     TV *__restrict__ part, int n, int64_t nn,
                                                     int64_t rows, int n_bands, int lines, int batch,
                                                     uint32_t *__restrict__ tickets)
{
    const int nbc = min(BC, batch);
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
        fwd_bundle<TM, TV, W, BC, BW>(d, idx, v0, v1, edge, d.horiz ? xT : x, part + int64_t(it.y) * rows, n, nn,
                                      stride, nbc, tq0, tq1);
    }
}

// Right-hand sides per fused chunk: the largest supported chunk that fits the
// batch and the operator's tuning limit.
inline int fwd_rhs_chunk(int batch, int limit)
{
    for (int c : {16, 8, 4})
        if (c <= batch && c <= limit) return c;
    return 1;
}

template <class TM, class TV, int W, int BC, int BW>
inline void fwd_wbc(const Op &op, const TV *x, const TV *xT, TV *y, int batch, hipStream_t s)
{
    const int64_t g = op.n_order < kPersistentBlocks ? op.n_order : kPersistentBlocks;
    const unsigned chunks = unsigned((batch + BC - 1) / BC);
    k_fwd<TM, TV, W, BC, BW><<<dim3(unsigned(g), chunks), 64 * W, 0, s>>>(
        op.fb, op.fb_order, op.n_order, op.f_idx, static_cast<const TM *>(op.f_v0),
        static_cast<const TM *>(op.f_v1), op.f_edge, x, xT ? xT : x, y, op.n, op.nn, op.rows, batch);
}

template <class TM, class TV, int BC, int BW>
inline void fwd_bcw(const Op &op, const TV *x, const TV *xT, TV *y, int batch, hipStream_t s)
{
    if (op.tune.fwd_waves == 2) fwd_wbc<TM, TV, 2, BC, BW>(op, x, xT, y, batch, s);
    else fwd_wbc<TM, TV, 4, BC, BW>(op, x, xT, y, batch, s);
}

template <class TM, class TV, int W, int BC, int BW>
inline void fwd_band_wbc(const Op &op, const BandSet &bs, const TV *x, const TV *xT, TV *y, TV *part,
                         int batch, hipStream_t s)
{
    // a multiple of 8 blocks, so that block i runs on XCD i % 8
    const int64_t g = bs.n_order < kPersistentBlocks ? (bs.n_order + 7) / 8 * 8 : kPersistentBlocks;
    uint32_t *tickets = nullptr;
    TV *unused = nullptr;
    fwd_scratch_layout(part, int64_t(bs.n_bands) * op.rows * BC, &tickets, &unused);
    k_ticket_reset<<<1, 64, 0, s>>>(tickets);
    k_fwd_band<TM, TV, W, BC, BW><<<dim3(unsigned(g), 1u), 64 * W, 0, s>>>(
        op.fb, bs.order, bs.n_order, op.f_idx, static_cast<const TM *>(op.f_v0),
        static_cast<const TM *>(op.f_v1), op.f_edge, x, xT ? xT : x, part, op.n, op.nn, op.rows, bs.n_bands,
        bs.lines, batch, tickets);
    k_fwd_band_sum<TV><<<dim3(unsigned((op.rows + 255) / 256), unsigned(batch)), 256, 0, s>>>(
        op.fb, part, y, op.rows, op.n_bins, op.bmap, bs.n_bands, bs.lines);
}

template <class TM, class TV, int BC, int BW>
inline void fwd_band_bcw(const Op &op, const BandSet &bs, const TV *x, const TV *xT, TV *y, TV *part,
                         int batch, hipStream_t s)
{
    if (op.tune.fwd_waves == 2) fwd_band_wbc<TM, TV, 2, BC, BW>(op, bs, x, xT, y, part, batch, s);
    else fwd_band_wbc<TM, TV, 4, BC, BW>(op, bs, x, xT, y, part, batch, s);
}

// Line-banded forward over chunks of bc images, one chunk after another (a
// chunk's band of images is what an XCD's L2 holds; chunks launched side by
// side would share it).  part holds one chunk's partials.
template <class TM, class TV, int BC, int BW>
inline void fwd_band_chunks(const Op &op, const BandSet &bs, const TV *x, const TV *xT, TV *y, TV *part,
                            int batch, hipStream_t s)
{
    for (int c0 = 0; c0 < batch; c0 += BC) {
        const int nb = batch - c0 < BC ? batch - c0 : BC;
        fwd_band_bcw<TM, TV, BC, BW>(op, bs, x + int64_t(c0) * op.nn, xT ? xT + int64_t(c0) * op.nn : nullptr,
                                     y + int64_t(c0) * op.rows, part, nb, s);
    }
}

template <class TM, class TV, int W, int C, int BW>
inline void fwd_pm_launch(const Op &op, const BandSet *bs, const TV *xp, const TV *xpT, TV *y, TV *part,
                          int nb, uint32_t *tickets, hipStream_t s)
{
    const TM *v0 = static_cast<const TM *>(op.f_v0), *v1 = static_cast<const TM *>(op.f_v1);
    if (bs) {
        // a multiple of 8 blocks, so that block i runs on XCD i % 8
        const int64_t g = bs->n_order < kPersistentBlocks ? (bs->n_order + 7) / 8 * 8 : kPersistentBlocks;
        k_ticket_reset<<<1, 64, 0, s>>>(tickets);
        k_fwd_pm_band<TM, TV, W, C, BW><<<unsigned(g), 64 * W, 0, s>>>(
            op.fb, bs->order, bs->n_order, op.f_idx, v0, v1, op.f_edge, xp, xpT, part, op.n, op.rows, bs->n_bands,
            bs->lines, nb, tickets);
        k_fwd_band_sum<TV><<<dim3(unsigned((op.rows + 255) / 256), unsigned(nb)), 256, 0, s>>>(
            op.fb, part, y, op.rows, op.n_bins, op.bmap, bs->n_bands, bs->lines);
    } else {
        const int64_t g = op.n_order < kPersistentBlocks ? op.n_order : kPersistentBlocks;
        k_fwd_pm<TM, TV, W, C, BW><<<unsigned(g), 64 * W, 0, s>>>(op.fb, op.fb_order, op.n_order, op.f_idx,
                                                                  v0, v1, op.f_edge, xp, xpT, y, op.n, op.rows, nb);
    }
}

// Forward over chunks of C images from pixel-major copies, one chunk after
// another: part holds the chunk's band partials (when banded), then, 256-byte
// aligned, the ticket counters, its pixel-major copy and (for operators with
// rays closer to horizontal) the copy in transposed pixel order.
template <class TM, class TV, int C, int BW>
inline void fwd_pm_chunks(const Op &op, const BandSet *bs, const TV *x, TV *y, TV *part, int batch,
                          hipStream_t s)
{
    uint32_t *tickets = nullptr;
    TV *xp = nullptr;
    fwd_scratch_layout(part, bs ? int64_t(bs->n_bands) * op.rows * C : 0, &tickets, &xp);
    TV *xpT = op.need_T ? xp + int64_t(C) * op.nn : nullptr;
    const unsigned t = unsigned((op.n + 15) / 16);
    for (int c0 = 0; c0 < batch; c0 += C) {
        const int nb = batch - c0 < C ? batch - c0 : C;
        k_pixel_major<TV, C><<<dim3(t, t), 256, 0, s>>>(x + int64_t(c0) * op.nn, xp, xpT, op.n, op.nn, nb);
        if (op.tune.fwd_waves == 2)
            fwd_pm_launch<TM, TV, 2, C, BW>(op, bs, xp, xpT ? xpT : xp, y + int64_t(c0) * op.rows, part, nb,
                                            tickets, s);
        else
            fwd_pm_launch<TM, TV, 4, C, BW>(op, bs, xp, xpT ? xpT : xp, y + int64_t(c0) * op.rows, part, nb,
                                            tickets, s);
    }
}

template <class TM, class TV, int BW>
int launch_fwd_bw(const Op &op, const TV *x, const TV *xT, TV *y, int batch, hipStream_t s, TV *part)
{
    if (op.sym) return launch_fwd_sym<TM, TV, BW>(op, x, xT, y, batch, s);
    const int bc = fwd_rhs_chunk(batch, op.tune.fwd_rhs);
    const BandSet *bs = part ? band_set_for(op, bc) : nullptr;
    if (part && fwd_pixel_major(op.tune.fwd_layout, bc)) {
        switch (bc) {
        case 16: fwd_pm_chunks<TM, TV, 16, BW>(op, bs, x, y, part, batch, s); break;
        case 8: fwd_pm_chunks<TM, TV, 8, BW>(op, bs, x, y, part, batch, s); break;
        default: fwd_pm_chunks<TM, TV, 4, BW>(op, bs, x, y, part, batch, s); break;
        }
        return check_launch("k_fwd_pm");
    }
    if (bs) {
        switch (bc) {
        case 16: fwd_band_chunks<TM, TV, 16, BW>(op, *bs, x, xT, y, part, batch, s); break;
        case 8: fwd_band_chunks<TM, TV, 8, BW>(op, *bs, x, xT, y, part, batch, s); break;
        case 4: fwd_band_chunks<TM, TV, 4, BW>(op, *bs, x, xT, y, part, batch, s); break;
        default: fwd_band_chunks<TM, TV, 1, BW>(op, *bs, x, xT, y, part, batch, s); break;
        }
        return check_launch("k_fwd_band");
    }
    switch (bc) {
    case 16: fwd_bcw<TM, TV, 16, BW>(op, x, xT, y, batch, s); break;
    case 8: fwd_bcw<TM, TV, 8, BW>(op, x, xT, y, batch, s); break;
    case 4: fwd_bcw<TM, TV, 4, BW>(op, x, xT, y, batch, s); break;
    default: fwd_bcw<TM, TV, 1, BW>(op, x, xT, y, batch, s); break;
    }
    return check_launch("k_fwd");
}

#define SCT_FWD_INST(BW)                                                                          \
    template int launch_fwd_bw<float, float, BW>(const Op &, const float *, const float *, float *, \
                                                 int, hipStream_t, float *);                       \
    template int launch_fwd_bw<double, double, BW>(const Op &, const double *, const double *,    \
                                                   double *, int, hipStream_t, double *);          \
    template int launch_fwd_bw<float, double, BW>(const Op &, const double *, const double *,     \
                                                  double *, int, hipStream_t, double *);

}  // namespace sct
