// Sparse products with the precomputed operator: y = MR x through the
// ray-bundle layout, x = (MR)^T y through the pixel-group layout, and the
// normal operator alpha R^T M^T M R + lambda K^T K + sigma I of eq:KKT,
// eq:PD_resolve and eq:SB_solve (Section 2) with the K^T K and sigma terms and
// the FP64 <x, Ax> partial sums fused into the adjoint's epilogue.
//
// Both products are bound by HBM bandwidth (2 flops per 5 bytes of stored
// matrix): no MFMA; the work is laid out so that the value/index streams are
// read with fully coalesced 64-lane loads and the gathers of the vector being
// multiplied touch a few cache lines per wave load.
#include "products.hpp"

#include <mutex>

namespace sct {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Single right-hand side version of k_adj below (kept separate: the fused
// multi-RHS form compiles to a slower loop for one image), over the same tile
// order.
template <class TM, class T, int W>
__global__ __launch_bounds__(64 * W) void k_adj1(const uint8_t *__restrict__ rel,
                                                const uint16_t *__restrict__ base,
                                                const TM *__restrict__ v0, const TM *__restrict__ v1,
                                                int64_t n_ag, int n_meas, int n_aq, int nb,
                                                const T *__restrict__ y, const T *__restrict__ x,
                                                T *__restrict__ out, T alpha, T lambda, T sigma,
                                                double *__restrict__ part, int n, int tiles,
                                                int64_t nn, int64_t rows,
                                                const int32_t *__restrict__ order, int64_t n_order)
{
    using Q = typename Quad<TM>::type;
    __shared__ T band[W * 4 * kAdjBand];
    __shared__ uint16_t bases[W * kAdjLanes];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t bat = blockIdx.y;
    const T *__restrict__ yb = y + bat * rows;
    const T *__restrict__ xb = x ? x + bat * nn : nullptr;
    const uint32_t *__restrict__ Rl = reinterpret_cast<const uint32_t *>(rel);
    const Q *__restrict__ A = reinterpret_cast<const Q *>(v0);
    const Q *__restrict__ Bv = reinterpret_cast<const Q *>(v1);
    double dsum = 0.0;   // this block's share of <x, out>, tiles in a fixed order
    // the tiles in the XCD-compact order of k_adj: a block visits the same
    // tiles as there, so one image's <x, out> partials equal a chunk's
    for (int64_t o = blockIdx.x; o < n_order; o += gridDim.x) {
        const int64_t g = order[o];
        if (g < 0) continue;   // padding entry (uniform per block)
        const T acc = adj_tile1<TM, T, W>(g, Rl, base, A, Bv, n_meas, n_aq, nb, yb, band, bases);
        if (wave == 0)
            dsum += adj_epilogue(g, lane, acc, xb, out + bat * nn, alpha, lambda, sigma, n, tiles);
    }
    if (part && wave == 0) {
        dsum = wave_sum(dsum);
        if (lane == 0) part[bat * gridDim.x + blockIdx.x] = dsum;
    }
}

// Adjoint of an operator whose adjoint is stored by symmetry (Op::sym_adj):
// pixel-group slots for the stored angles theta in [0, pi/4] only.  Pixel
// P = (px, py) meets the rays of a partner angle of theta with the lengths,
// bin for bin, with which its image Q meets the rays of theta:
//   pi - theta    (x -> -x):       Q = (n-1-px, py);
//   pi/2 - theta  (the transpose): Q = (py, px);
//   pi/2 + theta  (both):          Q = (py, n-1-px)
// (the maps of the forward's partner rays, inverted).  With n a multiple of
// 8 each map carries 8x8 tiles onto tiles and lanes onto lanes, so output
// tile g sums, per map, the stored quads of its source tile against the
// sinogram band of the partner angles (absent partners: zero band).  Lane l
// reads slot l of the source tile (whole 64-lane runs, as in adj_tile1) and
// keeps one sum per map for source pixel l; at the end of the tile the sums
// go through LDS to the output lanes they belong to.  A wave takes its share
// of the 4 * n_aq (map, quad) items; bases and partner angles are staged per
// chunk of quads in LDS.  The tiles of one orbit read the same slots and the
// tile order keeps them on one XCD at once, so the slots are read with plain
// loads and the later readers find them in L2.
template <class TM, class T, int W>
__global__ __launch_bounds__(64 * W) void k_adj1_sym(const uint8_t *__restrict__ rel,
                                                    const uint16_t *__restrict__ base,
                                                    const TM *__restrict__ v0, const TM *__restrict__ v1,
                                                    const int4 *__restrict__ partner, int n_rep, int n_aq,
                                                    int nb, const T *__restrict__ y, const T *__restrict__ x,
                                                    T *__restrict__ out, T alpha, T lambda, T sigma,
                                                    double *__restrict__ part, int n, int tiles, int64_t nn,
                                                    int64_t rows, const int32_t *__restrict__ order,
                                                    int64_t n_order)
{
    using Q = typename Quad<TM>::type;
    __shared__ T band[W][4 * kAdjBand];
    __shared__ uint16_t bases[W][kAdjLanes];
    __shared__ int32_t rowat[W][kAdjLanes];   // partner angle * nb, or -1
    __shared__ T red[W][4][64];               // per-map sums at their output lanes
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t bat = blockIdx.y;
    const T *__restrict__ yb = y + bat * rows;
    const T *__restrict__ xb = x ? x + bat * nn : nullptr;
    const uint32_t *__restrict__ Rl = reinterpret_cast<const uint32_t *>(rel);
    const Q *__restrict__ A = reinterpret_cast<const Q *>(v0);
    const Q *__restrict__ Bv = reinterpret_cast<const Q *>(v1);
    const int items = 4 * n_aq;
    const int q0 = (items * wave) / W, q1 = (items * (wave + 1)) / W;
    const int kk = lane >> 4, ee = lane & 15;   // this lane's band element
    // output lane of source lane (qy, qx) = (lane >> 3, lane & 7) per map
    const int sx = lane & 7, sy = lane >> 3;
    const int dest[4] = {lane, sy * 8 + (7 - sx), sx * 8 + sy, sx * 8 + (7 - sy)};
    T *__restrict__ my = band[wave];
    double dsum = 0.0;
    for (int64_t o = blockIdx.x; o < n_order; o += gridDim.x) {
        const int g = order[o];
        if (g < 0) continue;   // padding entry (uniform per block)
        const int tx = g % tiles, ty = g / tiles;
        T acc[4] = {T(0), T(0), T(0), T(0)};
        for (int c0 = q0; c0 < q1;) {
            const int mu = c0 / n_aq, aq0 = c0 % n_aq;   // wave-uniform
            const int nc = min(min(kBaseChunk, q1 - c0), n_aq - aq0);
            const int S = mu == 0 ? g
                        : mu == 1 ? ty * tiles + (tiles - 1 - tx)
                        : mu == 2 ? tx * tiles + ty
                                  : (tiles - 1 - tx) * tiles + ty;
            if (lane < 4 * nc) {
                const int a = 4 * aq0 + lane;
                int pa = -1;
                if (a < n_rep) {
                    const int4 p = partner[a];
                    pa = mu == 0 ? a : (mu == 1 ? p.x : (mu == 2 ? p.y : p.z));
                }
                bases[wave][lane] = base[(int64_t(S) * n_aq + aq0) * 4 + lane];
                rowat[wave][lane] = pa < 0 ? -1 : pa * nb;
            }
            __builtin_amdgcn_wave_barrier();
            T sum = T(0);
#pragma unroll 2
            for (int j = 0; j < nc; ++j) {
                const int64_t gq = int64_t(S) * n_aq + aq0 + j;
                const int ra = rowat[wave][4 * j + kk];
                const int b_band = min(int(bases[wave][4 * j + kk]) + ee, nb - 1);
                const T yv = ra >= 0 ? yb[int64_t(ra) + b_band] : T(0);
                const int64_t e = gq * kAdjLanes + lane;
                const uint32_t r4 = Rl[e];
                const Q a4 = A[e];
                const Q c4 = Bv[e];
                my[lane] = yv;
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int rb = int((r4 >> (8 * k)) & 0xffu);
                    sum = fma(T(a4[k]), my[k * kAdjBand + rb], sum);
                    sum = fma(T(c4[k]), my[k * kAdjBand + rb + 1], sum);
                }
                __builtin_amdgcn_wave_barrier();
            }
            if (mu == 0) acc[0] += sum;
            else if (mu == 1) acc[1] += sum;
            else if (mu == 2) acc[2] += sum;
            else acc[3] += sum;
            c0 += nc;
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) red[wave][m][dest[m]] = acc[m];
        __syncthreads();
        T tot = T(0);
        if (wave == 0) {
#pragma unroll
            for (int w = 0; w < W; ++w) {
#pragma unroll
                for (int m = 0; m < 4; ++m) tot += red[w][m][lane];
            }
        }
        __syncthreads();   // red is reused by the next tile
        if (wave == 0) dsum += adj_epilogue(g, lane, tot, xb, out + bat * nn, alpha, lambda, sigma, n, tiles);
    }
    if (part && wave == 0) {
        dsum = wave_sum(dsum);
        if (lane == 0) part[bat * gridDim.x + blockIdx.x] = dsum;
    }
}

// The same adjoint with one workgroup per tile orbit (k_adj1_sym's tiles of
// one orbit read the same slots, four times over).  Wave w takes the orbit's
// source tiles w, w + W, ... whole: it reads each of their stored slots once
// and applies the four maps to it, staging per quad the sinogram band of
// each map's partner angles (4 x 64 values) and forming four sums, one per
// map, for source pixel `lane`.  The sum of source s under map m is stored
// at [s][m][dest_m(lane)] in LDS (each written once); output tile t then adds
// its four sums, from sources src[t][0..3], in map order, and wave t % W
// applies the epilogue.
template <class TM, class T, int W>
__global__ __launch_bounds__(64 * W) void k_adj1_orb(const uint8_t *__restrict__ rel,
                                                    const uint16_t *__restrict__ base,
                                                    const TM *__restrict__ v0, const TM *__restrict__ v1,
                                                    const int4 *__restrict__ partner, int n_rep, int n_aq,
                                                    int nb, const T *__restrict__ y, const T *__restrict__ x,
                                                    T *__restrict__ out, T alpha, T lambda, T sigma,
                                                    double *__restrict__ part, int n, int tiles, int64_t nn,
                                                    int64_t rows, const AdjOrbit *__restrict__ orbs,
                                                    int64_t n_orb)
{
    using Q = typename Quad<TM>::type;
    __shared__ T band[W][4][4 * kAdjBand];
    __shared__ uint16_t bases[W][kAdjLanes];
    __shared__ int32_t rowat[W][4][kAdjLanes];   // partner angle * nb per map, or -1
    __shared__ T sums[8][4][64];                 // per source tile and map, at the output lanes
    __shared__ double dred[W];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t bat = blockIdx.y;
    const T *__restrict__ yb = y + bat * rows;
    const T *__restrict__ xb = x ? x + bat * nn : nullptr;
    const uint32_t *__restrict__ Rl = reinterpret_cast<const uint32_t *>(rel);
    const Q *__restrict__ A = reinterpret_cast<const Q *>(v0);
    const Q *__restrict__ Bv = reinterpret_cast<const Q *>(v1);
    const int kk = lane >> 4, ee = lane & 15;   // this lane's band element
    const int sx = lane & 7, sy = lane >> 3;
    const int d1 = sy * 8 + (7 - sx), d2 = sx * 8 + sy, d3 = sx * 8 + (7 - sy);
    double dsum = 0.0;
    for (int64_t o = blockIdx.x; o < n_orb; o += gridDim.x) {
        const AdjOrbit &ob = orbs[o];
        int k = 0;
#pragma unroll
        for (int t = 0; t < 8; ++t) k += ob.tile[t] >= 0 ? 1 : 0;
        for (int si = wave; si < k; si += W) {
            const int S = ob.tile[si];
            T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
            for (int aq0 = 0; aq0 < n_aq; aq0 += kBaseChunk) {
                const int nc = min(kBaseChunk, n_aq - aq0);
                if (lane < 4 * nc) {
                    const int a = 4 * aq0 + lane;
                    int4 p = make_int4(-1, -1, -1, -1);
                    if (a < n_rep) p = partner[a];
                    bases[wave][lane] = base[(int64_t(S) * n_aq + aq0) * 4 + lane];
                    rowat[wave][0][lane] = a < n_rep ? a * nb : -1;
                    rowat[wave][1][lane] = p.x < 0 ? -1 : p.x * nb;
                    rowat[wave][2][lane] = p.y < 0 ? -1 : p.y * nb;
                    rowat[wave][3][lane] = p.z < 0 ? -1 : p.z * nb;
                }
                __builtin_amdgcn_wave_barrier();
#pragma unroll 2
                for (int j = 0; j < nc; ++j) {
                    const int64_t gq = int64_t(S) * n_aq + aq0 + j;
                    const int bi = 4 * j + kk;
                    const int b_band = min(int(bases[wave][bi]) + ee, nb - 1);
                    T yv[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int ra = rowat[wave][m][bi];
                        yv[m] = ra >= 0 ? yb[int64_t(ra) + b_band] : T(0);
                    }
                    const int64_t e = gq * kAdjLanes + lane;
                    const uint32_t r4 = stream_load(Rl + e);
                    const Q a4 = stream_load(A + e);
                    const Q c4 = stream_load(Bv + e);
#pragma unroll
                    for (int m = 0; m < 4; ++m) band[wave][m][lane] = yv[m];
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int rb = q * kAdjBand + int((r4 >> (8 * q)) & 0xffu);
                        const T av = T(a4[q]), cv = T(c4[q]);
                        s0 = fma(av, band[wave][0][rb], s0);
                        s0 = fma(cv, band[wave][0][rb + 1], s0);
                        s1 = fma(av, band[wave][1][rb], s1);
                        s1 = fma(cv, band[wave][1][rb + 1], s1);
                        s2 = fma(av, band[wave][2][rb], s2);
                        s2 = fma(cv, band[wave][2][rb + 1], s2);
                        s3 = fma(av, band[wave][3][rb], s3);
                        s3 = fma(cv, band[wave][3][rb + 1], s3);
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
            sums[si][0][lane] = s0;
            sums[si][1][d1] = s1;
            sums[si][2][d2] = s2;
            sums[si][3][d3] = s3;
        }
        __syncthreads();
        for (int t = wave; t < k; t += W) {
            T tot = sums[ob.src[t][0]][0][lane];
            tot += sums[ob.src[t][1]][1][lane];
            tot += sums[ob.src[t][2]][2][lane];
            tot += sums[ob.src[t][3]][3][lane];
            dsum += adj_epilogue(ob.tile[t], lane, tot, xb, out + bat * nn, alpha, lambda, sigma, n, tiles);
        }
        __syncthreads();   // sums are rewritten by the next orbit
    }
    if (part) {
        dsum = wave_sum(dsum);
        if (lane == 0) dred[wave] = dsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double v = 0.0;
#pragma unroll
            for (int w = 0; w < W; ++w) v += dred[w];
            part[bat * gridDim.x + blockIdx.x] = v;
        }
    }
}

// Adjoint: one workgroup of W waves per 8x8 pixel tile (persistent loop over
// the tiles in `order`, the XCD-compact order: the tiles a workgroup on XCD x
// visits lie in one compact region of the image, so the sinogram bands the
// XCD's concurrent tiles read stay in its L2 for every image of the chunk).  Wave w sums its share of the measured-angle quads for the tile's
// 64 pixels.  Per quad it stages the tile's sinogram band (16 bins from the
// tile's base bin, for each of the 4 angles: exactly one 64-lane load) in LDS
// and reads the pixel's two bins from there, so the vector-memory pipeline
// only carries the three matrix streams and the band.  The wave shares are
// added in wave order, and wave 0 applies the epilogue
// out = alpha*acc + lambda*(K^T K x) + sigma*x and the FP64 partial <x, out>.
// Several right-hand sides: blockIdx.y selects a chunk of up to BC sinograms
// that share every matrix load; each gets its own band and accumulator.
template <class TM, class T, int W, int BC>
__global__ __launch_bounds__(64 * W) void k_adj(const uint8_t *__restrict__ rel,
                                                const uint16_t *__restrict__ base,
                                                const TM *__restrict__ v0, const TM *__restrict__ v1,
                                                int64_t n_ag, int n_meas, int n_aq, int nb,
                                                const T *__restrict__ y, const T *__restrict__ x,
                                                T *__restrict__ out, T alpha, T lambda, T sigma,
                                                double *__restrict__ part, int n, int tiles,
                                                int64_t nn, int64_t rows, int batch,
                                                const int32_t *__restrict__ order, int64_t n_order)
{
    using Q = typename Quad<TM>::type;
    __shared__ T band[W][BC][4 * kAdjBand];
    __shared__ uint16_t bases[W][kAdjLanes];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int b0 = int(blockIdx.y) * BC;
    const int nbc = min(BC, batch - b0);
    const T *__restrict__ yb = y + int64_t(b0) * rows;
    const int q0 = (n_aq * wave) / W, q1 = (n_aq * (wave + 1)) / W;
    const uint32_t *__restrict__ Rl = reinterpret_cast<const uint32_t *>(rel);
    const Q *__restrict__ A = reinterpret_cast<const Q *>(v0);
    const Q *__restrict__ Bv = reinterpret_cast<const Q *>(v1);
    const int kk = lane >> 4, ee = lane & 15;   // this lane's band element
    double dsum[BC];                            // this block's share of <x, out>
#pragma unroll
    for (int c = 0; c < BC; ++c) dsum[c] = 0.0;
    for (int64_t o = blockIdx.x; o < n_order; o += gridDim.x) {
        const int64_t g = order[o];
        if (g < 0) continue;   // padding entry (uniform per block)
        T acc[BC];
#pragma unroll
        for (int c = 0; c < BC; ++c) acc[c] = T(0);
        for (int c0 = q0; c0 < q1; c0 += kBaseChunk) {
            const int nc = min(kBaseChunk, q1 - c0);
            if (lane < 4 * nc) bases[wave][lane] = base[(g * n_aq + c0) * 4 + lane];
            __builtin_amdgcn_wave_barrier();
#pragma unroll 2
            for (int j = 0; j < nc; ++j) {
                const int aq = c0 + j;
                const int64_t gq = g * n_aq + aq;
                const int a_band = min(4 * aq + kk, n_meas - 1);
                const int64_t band_at =
                    int64_t(a_band) * nb + min(int(bases[wave][4 * j + kk]) + ee, nb - 1);
                T yv[BC];
#pragma unroll
                for (int c = 0; c < BC; ++c)
                    if (BC == 1 || c < nbc) yv[c] = yb[int64_t(c) * rows + band_at];
                const int64_t e = gq * kAdjLanes + lane;
                const uint32_t r4 = stream_load(Rl + e);
                const Q a4 = stream_load(A + e);
                const Q c4 = stream_load(Bv + e);
#pragma unroll
                for (int c = 0; c < BC; ++c)
                    if (BC == 1 || c < nbc) band[wave][c][lane] = yv[c];
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int rb = k * kAdjBand + int((r4 >> (8 * k)) & 0xffu);
#pragma unroll
                    for (int c = 0; c < BC; ++c) {
                        if (BC == 1 || c < nbc) {
                            acc[c] = fma(T(a4[k]), band[wave][c][rb], acc[c]);
                            acc[c] = fma(T(c4[k]), band[wave][c][rb + 1], acc[c]);
                        }
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        if constexpr (W > 1) {
            __shared__ T red[W][BC][64];
#pragma unroll
            for (int c = 0; c < BC; ++c) red[wave][c][lane] = acc[c];
            __syncthreads();
            if (wave == 0) {
#pragma unroll
                for (int c = 0; c < BC; ++c) {
                    acc[c] = red[0][c][lane];
#pragma unroll
                    for (int w = 1; w < W; ++w) acc[c] += red[w][c][lane];
                }
            }
            __syncthreads();   // red is reused by the next tile
        }
        if (wave == 0) {
#pragma unroll
            for (int c = 0; c < BC; ++c) {
                if (BC == 1 || c < nbc)
                    dsum[c] += adj_epilogue(g, lane, acc[c], x ? x + int64_t(b0 + c) * nn : nullptr,
                                            out + int64_t(b0 + c) * nn, alpha, lambda, sigma, n,
                                            tiles);
            }
        }
    }
    if (part && wave == 0) {
#pragma unroll
        for (int c = 0; c < BC; ++c) {
            const double v = wave_sum(dsum[c]);
            if (c < nbc && lane == 0) part[int64_t(b0 + c) * gridDim.x + blockIdx.x] = v;
        }
    }
}

// Pixel-major copy of a chunk of nb sinograms: dst[i*C + c] = src[c*count + i]
// for c < nb, 0 for nb <= c < C, through a tile of 64 measurements x C in LDS
// (reads along i, writes along c).
template <class T, int C>
__global__ __launch_bounds__(256) void k_chunk_pm(const T *__restrict__ src, T *__restrict__ dst,
                                                  int64_t count, int nb)
{
    __shared__ T tile[C][65];
    const int64_t i0 = int64_t(blockIdx.x) * 64;
    for (int k = threadIdx.x; k < 64 * C; k += 256) {
        const int c = k / 64, i = k % 64;
        tile[c][i] = (c < nb && i0 + i < count) ? src[int64_t(c) * count + i0 + i] : T(0);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 64 * C; k += 256) {
        const int c = k % C, i = k / C;
        if (i0 + i < count) dst[(i0 + i) * C + c] = tile[c][i];
    }
}

// k_adj for one chunk of C sinograms given pixel-major (ypm[ray][c], the
// slots of absent images zero): each lane stages its band element for all C
// images with C / VW 16-byte loads and LDS writes, and reads a slot's two
// bins for 4 FP32 or 2 FP64 images per 16-byte LDS read.  The per-image
// staging of k_adj moves a 64-byte band run per angle and image through the
// L1, most of a 128-byte line; here one angle's band for the chunk is
// 16 x C x 4 or 8 contiguous bytes.  Tile order, wave split, summation order
// per image and the epilogue are those of k_adj.
template <class TM, class T, int W, int C>
__global__ __launch_bounds__(64 * W) void k_adj_pm(const uint8_t *__restrict__ rel,
                                                   const uint16_t *__restrict__ base,
                                                   const TM *__restrict__ v0, const TM *__restrict__ v1,
                                                   int n_meas, int n_aq, int nb, const T *__restrict__ ypm,
                                                   const T *__restrict__ x, T *__restrict__ out, T alpha,
                                                   T lambda, T sigma, double *__restrict__ part, int n,
                                                   int tiles, int64_t nn, int nbc,
                                                   const int32_t *__restrict__ order, int64_t n_order)
{
    using Q = typename Quad<TM>::type;
    using V = typename Vec16<T>::type;
    constexpr int VW = 16 / int(sizeof(T)), NG = C / VW;
    __shared__ V band[W][4 * kAdjBand][NG];
    __shared__ uint16_t bases[W][kAdjLanes];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int q0 = (n_aq * wave) / W, q1 = (n_aq * (wave + 1)) / W;
    const uint32_t *__restrict__ Rl = reinterpret_cast<const uint32_t *>(rel);
    const Q *__restrict__ A = reinterpret_cast<const Q *>(v0);
    const Q *__restrict__ Bv = reinterpret_cast<const Q *>(v1);
    const V *__restrict__ yv16 = reinterpret_cast<const V *>(ypm);
    const int kk = lane >> 4, ee = lane & 15;   // this lane's band element
    double dsum[C];                             // this block's share of <x, out>
#pragma unroll
    for (int c = 0; c < C; ++c) dsum[c] = 0.0;
    for (int64_t o = blockIdx.x; o < n_order; o += gridDim.x) {
        const int64_t g = order[o];
        if (g < 0) continue;   // padding entry (uniform per block)
        T acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = T(0);
        for (int c0 = q0; c0 < q1; c0 += kBaseChunk) {
            const int nc = min(kBaseChunk, q1 - c0);
            if (lane < 4 * nc) bases[wave][lane] = base[(g * n_aq + c0) * 4 + lane];
            __builtin_amdgcn_wave_barrier();
#pragma unroll 2
            for (int j = 0; j < nc; ++j) {
                const int aq = c0 + j;
                const int64_t gq = g * n_aq + aq;
                const int a_band = min(4 * aq + kk, n_meas - 1);
                const int64_t band_at =
                    int64_t(a_band) * nb + min(int(bases[wave][4 * j + kk]) + ee, nb - 1);
                V yv[NG];
#pragma unroll
                for (int h = 0; h < NG; ++h) yv[h] = yv16[band_at * NG + h];
                const int64_t e = gq * kAdjLanes + lane;
                const uint32_t r4 = stream_load(Rl + e);
                const Q a4 = stream_load(A + e);
                const Q c4 = stream_load(Bv + e);
#pragma unroll
                for (int h = 0; h < NG; ++h) band[wave][lane][h] = yv[h];
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int rb = k * kAdjBand + int((r4 >> (8 * k)) & 0xffu);
                    const T a = T(a4[k]), b = T(c4[k]);
#pragma unroll
                    for (int h = 0; h < NG; ++h) {
                        const V u = band[wave][rb][h], w = band[wave][rb + 1][h];
#pragma unroll
                        for (int v = 0; v < VW; ++v) {
                            acc[h * VW + v] = fma(a, u[v], acc[h * VW + v]);
                            acc[h * VW + v] = fma(b, w[v], acc[h * VW + v]);
                        }
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        if constexpr (W > 1) {
            __shared__ T red[W][C][64];
#pragma unroll
            for (int c = 0; c < C; ++c) red[wave][c][lane] = acc[c];
            __syncthreads();
            if (wave == 0) {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    acc[c] = red[0][c][lane];
#pragma unroll
                    for (int w = 1; w < W; ++w) acc[c] += red[w][c][lane];
                }
            }
            __syncthreads();   // red is reused by the next tile
        }
        if (wave == 0) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (c < nbc)
                    dsum[c] += adj_epilogue(g, lane, acc[c], x ? x + int64_t(c) * nn : nullptr,
                                            out + int64_t(c) * nn, alpha, lambda, sigma, n, tiles);
            }
        }
    }
    if (part && wave == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const double v = wave_sum(dsum[c]);
            if (c < nbc && lane == 0) part[int64_t(c) * gridDim.x + blockIdx.x] = v;
        }
    }
}

// dst[b] = sum_i part[b][i], in a fixed order (one block per b).
__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ part,
                                                      int64_t count, double *__restrict__ dst)
{
    __shared__ double red[256];
    const int64_t b = blockIdx.x;
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256) v += part[b * count + i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) dst[b] = red[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static int check_grid_y(int batch)
{
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    return RADON_OK;
}

template <class TV>
int launch_transpose(const Op &op, const TV *x, TV *xT, int batch, hipStream_t s)
{
    SCT_TRY(check_grid_y(batch));
    const unsigned t = unsigned((op.n + 31) / 32);
    k_transpose<TV><<<dim3(t, t, unsigned(batch)), dim3(32, 8), 0, s>>>(x, xT, op.n, op.nn);
    return check_launch("k_transpose");
}

// Right-hand sides per fused chunk: the largest supported chunk that fits the
// batch and the operator's tuning limit.
static int rhs_chunk(int batch, int limit)
{
    for (int c : {16, 8, 4})
        if (c <= batch && c <= limit) return c;
    return 1;
}

int fwd_chunk(const Op &op, int batch) { return rhs_chunk(batch, op.tune.fwd_rhs); }

const BandSet *band_set_lines(const Op &op, int bc, int lines)
{
    if (lines > 0) {
        for (const BandSet &b : op.bands)
            if (b.n_bands > 0 && b.lines == lines) return &b;
        return nullptr;   // not built (radon_set_tuning only accepts built heights)
    }
    const int64_t line = int64_t(op.n) * op.vsize;
    if (op.n < kBandMinN && int64_t(bc) * op.n * line <= kBandBudget) return nullptr;
    const BandSet *last = nullptr;
    for (const BandSet &b : op.bands) {
        if (b.n_bands <= 0) continue;
        if (int64_t(bc) * b.lines * line <= kBandBudget) return &b;
        last = &b;
    }
    return last;   // the lowest bands even where a chunk's band overflows the budget
}

int64_t fwd_scratch_elems(const Op &op, int bc, int nb, int layout, int lines)
{
    const BandSet *b = band_set_lines(op, bc, lines);
    const bool pm = fwd_pixel_major(layout, bc);
    int64_t e = b ? int64_t(b->n_bands) * op.rows * nb : 0;
    if (b || pm) e += kTicketSlack;
    if (pm) e += kPixelMajorSlack + int64_t(op.need_T ? 2 : 1) * bc * op.nn;
    return e;
}

// One chunk's band partials and pixel-major copies (chunks run one after
// another).
int64_t fwd_part_elems(const Op &op, int batch)
{
    const int bc = fwd_chunk(op, batch);
    return fwd_scratch_elems(op, bc, batch < bc ? batch : bc, op.tune.fwd_layout, op.tune.fwd_lines);
}

template <class TM, class TV>
int launch_fwd(const Op &op, const TV *x, const TV *xT, TV *y, int batch, hipStream_t s, TV *part)
{
    SCT_TRY(check_grid_y(batch));
    switch (op.bw) {
    case 64: return launch_fwd_bw<TM, TV, 64>(op, x, xT, y, batch, s, part);
    case 32: return launch_fwd_bw<TM, TV, 32>(op, x, xT, y, batch, s, part);
    default: return launch_fwd_bw<TM, TV, 16>(op, x, xT, y, batch, s, part);
    }
}

// The adjoint stored by symmetry with one workgroup per tile orbit.
static bool adj_by_orbit(const Op &op) { return op.sym_adj && op.a_orb && op.tune.adj_layout == 1; }

int adj_blocks(const Op &op)
{
    const int64_t items = adj_by_orbit(op) ? op.n_orb : op.n_ag;
    return int(items < kPersistentBlocks ? items : kPersistentBlocks);
}

static int adj_waves(const Op &op)
{
    if (op.tune.adj_waves == 1 || op.tune.adj_waves == 2 || op.tune.adj_waves == 4) return op.tune.adj_waves;
    return adj_waves_for(op.n_meas);
}

template <class TM, class TV, int W, int BC>
static void adj_wbc(const Op &op, const TV *y, const TV *x, TV *out, TV al, TV la, TV si,
                    double *part, int batch, hipStream_t s, TV *scratch)
{
    const dim3 grid(unsigned(adj_blocks(op)), unsigned((batch + BC - 1) / BC));
    const TM *a0 = static_cast<const TM *>(op.a_v0), *a1 = static_cast<const TM *>(op.a_v1);
    if constexpr (BC > 1) {
        if (scratch && op.tune.adj_layout == 1) {
            // chunks one after another, each from its pixel-major copy
            const uintptr_t a = (reinterpret_cast<uintptr_t>(scratch) + 15) & ~uintptr_t(15);
            TV *ypm = reinterpret_cast<TV *>(a);
            const unsigned G = grid.x;
            for (int c0 = 0; c0 < batch; c0 += BC) {
                const int nb = batch - c0 < BC ? batch - c0 : BC;
                k_chunk_pm<TV, BC><<<unsigned((op.rows + 63) / 64), 256, 0, s>>>(y + int64_t(c0) * op.rows, ypm,
                                                                                 op.rows, nb);
                k_adj_pm<TM, TV, W, BC><<<dim3(G, 1u), 64 * W, 0, s>>>(
                    op.a_rel, op.a_base, a0, a1, op.n_meas, op.n_aq, op.n_bins, ypm,
                    x ? x + int64_t(c0) * op.nn : nullptr, out + int64_t(c0) * op.nn, al, la, si,
                    part ? part + int64_t(c0) * G : nullptr, op.n, op.tiles, op.nn, nb, op.a_order,
                    op.n_a_order);
            }
            return;
        }
    }
    if constexpr (BC == 1)
        k_adj1<TM, TV, W><<<grid, 64 * W, 0, s>>>(op.a_rel, op.a_base, a0, a1, op.n_ag, op.n_meas,
                                                 op.n_aq, op.n_bins, y, x, out, al, la, si, part,
                                                 op.n, op.tiles, op.nn, op.rows, op.a_order,
                                                 op.n_a_order);
    else {
        // chunks one after another: a chunk's sinograms share the XCDs' L2
        const unsigned G = grid.x;
        for (int c0 = 0; c0 < batch; c0 += BC) {
            const int nb = batch - c0 < BC ? batch - c0 : BC;
            k_adj<TM, TV, W, BC><<<dim3(G, 1u), 64 * W, 0, s>>>(
                op.a_rel, op.a_base, a0, a1, op.n_ag, op.n_meas, op.n_aq, op.n_bins,
                y + int64_t(c0) * op.rows, x ? x + int64_t(c0) * op.nn : nullptr,
                out + int64_t(c0) * op.nn, al, la, si, part ? part + int64_t(c0) * G : nullptr, op.n,
                op.tiles, op.nn, op.rows, nb, op.a_order, op.n_a_order);
        }
    }
}

// Adjoint stored by symmetry: one image per blockIdx.y.
template <class TM, class TV>
static void adj_sym(const Op &op, const TV *y, const TV *x, TV *out, TV al, TV la, TV si, double *part,
                    int batch, hipStream_t s)
{
    const dim3 grid(unsigned(adj_blocks(op)), unsigned(batch));
    const TM *a0 = static_cast<const TM *>(op.a_v0), *a1 = static_cast<const TM *>(op.a_v1);
    if (adj_by_orbit(op)) {
        // 2 x adj_waves waves per orbit (default 8: one per source tile)
#define SCT_ORB(W)                                                                                     \
    k_adj1_orb<TM, TV, W><<<grid, 64 * W, 0, s>>>(op.a_rel, op.a_base, a0, a1, op.f_partner, op.n_rep, \
                                                  op.n_aq, op.n_bins, y, x, out, al, la, si, part, op.n, \
                                                  op.tiles, op.nn, op.rows, op.a_orb, op.n_orb)
        if (op.tune.adj_waves == 1) SCT_ORB(2);
        else if (op.tune.adj_waves == 2) SCT_ORB(4);
        else SCT_ORB(8);
#undef SCT_ORB
        return;
    }
#define SCT_SYM(W)                                                                                    \
    k_adj1_sym<TM, TV, W><<<grid, 64 * W, 0, s>>>(op.a_rel, op.a_base, a0, a1, op.f_partner, op.n_rep, \
                                                  op.n_aq, op.n_bins, y, x, out, al, la, si, part, op.n, \
                                                  op.tiles, op.nn, op.rows, op.a_order, op.n_a_order)
    // default: about 12 or more (map, quad) items per wave
    const int items = 4 * op.n_aq;
    const int w = op.tune.adj_waves == 1 || op.tune.adj_waves == 2 || op.tune.adj_waves == 4
                      ? op.tune.adj_waves
                      : (items >= 48 ? 4 : (items >= 24 ? 2 : 1));
    if (w == 4) SCT_SYM(4);
    else if (w == 2) SCT_SYM(2);
    else SCT_SYM(1);
#undef SCT_SYM
}

template <class TM, class TV, int BC>
static void adj_bc(const Op &op, const TV *y, const TV *x, TV *out, TV al, TV la, TV si,
                   double *part, int batch, hipStream_t s, TV *scratch)
{
    switch (adj_waves(op)) {
    case 4: adj_wbc<TM, TV, 4, BC>(op, y, x, out, al, la, si, part, batch, s, scratch); break;
    case 2: adj_wbc<TM, TV, 2, BC>(op, y, x, out, al, la, si, part, batch, s, scratch); break;
    default: adj_wbc<TM, TV, 1, BC>(op, y, x, out, al, la, si, part, batch, s, scratch); break;
    }
}

int64_t adj_scratch_elems(const Op &op, int batch)
{
    const int bc = rhs_chunk(batch, op.tune.adj_rhs);
    if (op.sym_adj || op.tune.adj_layout != 1 || bc < 4) return 0;
    return kPixelMajorSlack + int64_t(bc) * op.rows;
}

int64_t prod_scratch_elems(const Op &op, int batch)
{
    const int64_t f = fwd_part_elems(op, batch), a = adj_scratch_elems(op, batch);
    return f > a ? f : a;
}

template <class TM, class TV>
int launch_adj(const Op &op, const TV *y, const TV *x, TV *out, double alpha, double lambda,
               double sigma, double *part, int batch, hipStream_t s, TV *scratch)
{
    SCT_TRY(check_grid_y(batch));
    const TV al = TV(alpha), la = TV(lambda), si = TV(sigma);
    if (op.sym_adj) {
        adj_sym<TM, TV>(op, y, x, out, al, la, si, part, batch, s);
        return check_launch("k_adj1_sym");
    }
    switch (rhs_chunk(batch, op.tune.adj_rhs)) {
    case 16: adj_bc<TM, TV, 16>(op, y, x, out, al, la, si, part, batch, s, scratch); break;
    case 8: adj_bc<TM, TV, 8>(op, y, x, out, al, la, si, part, batch, s, scratch); break;
    case 4: adj_bc<TM, TV, 4>(op, y, x, out, al, la, si, part, batch, s, scratch); break;
    default: adj_bc<TM, TV, 1>(op, y, x, out, al, la, si, part, batch, s, scratch); break;
    }
    return check_launch("k_adj");
}

int launch_sum_partials(const double *part, int64_t count, double *dst, int batch, hipStream_t s)
{
    k_sum_partials<<<unsigned(batch), 256, 0, s>>>(part, count, dst);
    return check_launch("k_sum_partials");
}

template int launch_transpose<float>(const Op &, const float *, float *, int, hipStream_t);
template int launch_transpose<double>(const Op &, const double *, double *, int, hipStream_t);
#define SCT_INST(TM, TV)                                                                          \
    template int launch_fwd<TM, TV>(const Op &, const TV *, const TV *, TV *, int, hipStream_t,   \
                                    TV *);                                                        \
    template int launch_adj<TM, TV>(const Op &, const TV *, const TV *, TV *, double, double,     \
                                    double, double *, int, hipStream_t, TV *);
SCT_INST(float, float)
SCT_INST(double, double)
SCT_INST(float, double)
#undef SCT_INST

// ---------------------------------------------------------------------------
// workspace sizes
// ---------------------------------------------------------------------------

static int64_t fwd_ws_bytes(const Op &op, int batch)
{
    Carver c(nullptr);
    if (op.need_T) c.take<char>(int64_t(op.vsize) * op.nn * batch);
    c.take<char>(int64_t(op.vsize) * fwd_part_elems(op, batch));
    return c.used;
}

// dst = src between [batch][count] and [count][batch] through a 32 x 32
// tile: blockIdx.x covers 32 elements of count, blockIdx.y 32 of the batch;
// both the read and the write run along the contiguous index.
template <class T>
__global__ __launch_bounds__(256) void k_relayout(const T *__restrict__ src, T *__restrict__ dst,
                                                  int64_t count, int batch, int to_pixel)
{
    __shared__ T tile[32][33];
    const int64_t i0 = int64_t(blockIdx.x) * 32;
    const int b0 = blockIdx.y * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;
    if (to_pixel) {
        for (int k = ty; k < 32; k += 8) {
            const int b = b0 + k;
            const int64_t i = i0 + tx;
            if (b < batch && i < count) tile[k][tx] = src[int64_t(b) * count + i];
        }
        __syncthreads();
        for (int k = ty; k < 32; k += 8) {
            const int64_t i = i0 + k;
            const int b = b0 + tx;
            if (i < count && b < batch) dst[i * batch + b] = tile[tx][k];
        }
    } else {
        for (int k = ty; k < 32; k += 8) {
            const int64_t i = i0 + k;
            const int b = b0 + tx;
            if (i < count && b < batch) tile[k][tx] = src[i * batch + b];
        }
        __syncthreads();
        for (int k = ty; k < 32; k += 8) {
            const int b = b0 + k;
            const int64_t i = i0 + tx;
            if (b < batch && i < count) dst[int64_t(b) * count + i] = tile[tx][k];
        }
    }
}

template <class TV>
int launch_relayout(const TV *src, TV *dst, int64_t count, int batch, bool to_pixel, hipStream_t s)
{
    const int64_t gx = (count + 31) / 32;
    if (gx > 0x7fffffffll) return set_error(RADON_EUNSUPPORTED, "%lld elements per image are too many", (long long)count);
    const dim3 grid(unsigned(gx), unsigned((batch + 31) / 32));
    k_relayout<TV><<<grid, dim3(32, 8), 0, s>>>(src, dst, count, batch, to_pixel ? 1 : 0);
    return check_launch("k_relayout");
}
template int launch_relayout<float>(const float *, float *, int64_t, int, bool, hipStream_t);
template int launch_relayout<double>(const double *, double *, int64_t, int, bool, hipStream_t);

int check_layout(int32_t layout)
{
    if (layout != RADON_LAYOUT_IMAGE && layout != RADON_LAYOUT_PIXEL)
        return set_error(RADON_EINVAL, "layout must be RADON_LAYOUT_IMAGE or RADON_LAYOUT_PIXEL (got %d)", layout);
    return RADON_OK;
}

int64_t pixel_layout_extra(const Op &op, int which, int batch)
{
    if (batch <= 1) return 0;
    Carver c(nullptr);
    const int64_t img = int64_t(op.vsize) * op.nn * batch, sino = int64_t(op.vsize) * op.rows * batch;
    switch (which) {
    case RADON_WS_FWD:
    case RADON_WS_ADJ:
    case RADON_WS_SB:
        c.take<char>(img);
        c.take<char>(sino);
        break;
    default:   // normal operator, CG: input and output images
        c.take<char>(img);
        c.take<char>(img);
        break;
    }
    return c.used + 256;   // the relay buffers start at a 256-byte boundary after the workspace
}

// The relay buffers of a pixel-major call: after `base` bytes of ws, 256-byte
// aligned; first of `n0` elements, second of `n1`.
template <class TV>
void relay_buffers(void *ws, int64_t base, int64_t n0, int64_t n1, TV **b0, TV **b1)
{
    char *p = static_cast<char *>(ws) + ((base + 255) & ~int64_t(255));
    Carver c(p);
    *b0 = c.take<TV>(n0);
    *b1 = c.take<TV>(n1);
}
template void relay_buffers<float>(void *, int64_t, int64_t, int64_t, float **, float **);
template void relay_buffers<double>(void *, int64_t, int64_t, int64_t, double **, double **);

static int64_t normal_ws_bytes(const Op &op, int batch)
{
    Carver c(nullptr);
    if (op.need_T) c.take<char>(int64_t(op.vsize) * op.nn * batch);
    c.take<char>(int64_t(op.vsize) * op.rows * batch);
    c.take<double>(op.n_ag * batch);
    c.take<char>(int64_t(op.vsize) * prod_scratch_elems(op, batch));
    return c.used;
}

static int64_t adj_ws_bytes(const Op &op, int batch) { return int64_t(op.vsize) * adj_scratch_elems(op, batch); }

int64_t cg_ws_bytes(const Op &op, int batch);   // solve.hip
int64_t sb_ws_bytes(const Op &op, int batch);   // solve.hip
int64_t pd_ws_bytes(const Op &op, int batch);   // solve.hip
int64_t tune_ws_bytes(const Op &op, int batch); // tune.hip

}  // namespace sct

using namespace sct;

extern "C" int64_t radon_workspace_bytes(const radon_op *p, int32_t which, int32_t batch)
{
    clear_error();
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    const Op &op = *as_op(p);
    const bool pixel = (which & RADON_WS_PIXEL_LAYOUT) != 0;
    const int kind = which & ~RADON_WS_PIXEL_LAYOUT;
    if (pixel && (kind == RADON_WS_PD || kind == RADON_WS_TUNE))
        return set_error(RADON_EINVAL, "workspace kind %d has no pixel-major form", kind);
    const int64_t extra = pixel ? pixel_layout_extra(op, kind, batch) : 0;
    switch (kind) {
    case RADON_WS_FWD: return fwd_ws_bytes(op, batch) + extra;
    case RADON_WS_ADJ: return adj_ws_bytes(op, batch) + extra;
    case RADON_WS_NORMAL: return normal_ws_bytes(op, batch) + extra;
    case RADON_WS_CG: return cg_ws_bytes(op, batch) + extra;
    case RADON_WS_SB: return sb_ws_bytes(op, batch) + extra;
    case RADON_WS_PD: return pd_ws_bytes(op, batch);
    case RADON_WS_TUNE: return tune_ws_bytes(op, batch);
    default: return set_error(RADON_EINVAL, "unknown workspace kind %d", which);
    }
}

// The image-major forward with its workspace.
static int fwd_into(const Op &op, const void *x, void *y, int batch, void *ws, hipStream_t s)
{
    return dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        Carver c(ws);
        const TV *xx = static_cast<const TV *>(x);
        TV *xT = nullptr;
        if (op.need_T) {
            xT = c.take<TV>(op.nn * batch);
            SCT_TRY(launch_transpose<TV>(op, xx, xT, batch, s));
        }
        const int64_t pe = fwd_part_elems(op, batch);
        TV *part = c.take<TV>(pe);
        return launch_fwd<TM, TV>(op, xx, xT, static_cast<TV *>(y), batch, s, pe ? part : nullptr);
    });
}

extern "C" int radon_fwd(const radon_op *p, const void *x, void *y, int32_t batch, int32_t layout,
                         void *ws, int64_t ws_bytes, void *stream)
{
    clear_error();
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    SCT_TRY(check_layout(layout));
    if (!x || !y) return set_error(RADON_EINVAL, "x and y must be non-NULL");
    const Op &op = *as_op(p);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t base = fwd_ws_bytes(op, batch);
    if (!relays(layout, batch)) {
        SCT_TRY(check_ws(ws, ws_bytes, base, "radon_fwd"));
        return fwd_into(op, x, y, batch, ws, s);
    }
    SCT_TRY(check_ws(ws, ws_bytes, base + pixel_layout_extra(op, RADON_WS_FWD, batch), "radon_fwd"));
    return dispatch(op, [&](auto *, auto *tv) {
        using TV = std::remove_pointer_t<decltype(tv)>;
        TV *xi = nullptr, *yi = nullptr;
        relay_buffers<TV>(ws, base, op.nn * batch, op.rows * batch, &xi, &yi);
        SCT_TRY(launch_relayout<TV>(static_cast<const TV *>(x), xi, op.nn, batch, false, s));
        SCT_TRY(fwd_into(op, xi, yi, batch, ws, s));
        return launch_relayout<TV>(yi, static_cast<TV *>(y), op.rows, batch, true, s);
    });
}

extern "C" int radon_fwd_xt(const radon_op *p, const void *x, const void *xT, void *y,
                            int32_t batch, void *stream)
{
    clear_error();
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    if (!x || !y) return set_error(RADON_EINVAL, "x and y must be non-NULL");
    const Op &op = *as_op(p);
    if (op.need_T && !xT)
        return set_error(RADON_EINVAL, "this geometry gathers from the transposed image: xT is required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        return launch_fwd<TM, TV>(op, static_cast<const TV *>(x), static_cast<const TV *>(xT),
                                  static_cast<TV *>(y), batch, s);
    });
}

extern "C" int radon_adj(const radon_op *p, const void *y, void *x, int32_t batch, int32_t layout,
                         void *ws, int64_t ws_bytes, void *stream)
{
    clear_error();
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    SCT_TRY(check_layout(layout));
    if (!x || !y) return set_error(RADON_EINVAL, "x and y must be non-NULL");
    const Op &op = *as_op(p);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t base = adj_ws_bytes(op, batch);
    if (!relays(layout, batch)) {
        // the workspace is optional here: without it every sinogram of a
        // chunk is staged on its own
        const bool scr = base > 0 && ws && ws_bytes >= base;
        return dispatch(op, [&](auto *tm, auto *tv) {
            SCT_TYPES(tm, tv);
            return launch_adj<TM, TV>(op, static_cast<const TV *>(y), nullptr, static_cast<TV *>(x), 1.0,
                                      0.0, 0.0, nullptr, batch, s, scr ? static_cast<TV *>(ws) : nullptr);
        });
    }
    SCT_TRY(check_ws(ws, ws_bytes, base + pixel_layout_extra(op, RADON_WS_ADJ, batch), "radon_adj"));
    return dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        TV *xi = nullptr, *yi = nullptr;
        relay_buffers<TV>(ws, base, op.nn * batch, op.rows * batch, &xi, &yi);
        SCT_TRY(launch_relayout<TV>(static_cast<const TV *>(y), yi, op.rows, batch, false, s));
        SCT_TRY((launch_adj<TM, TV>(op, yi, nullptr, xi, 1.0, 0.0, 0.0, nullptr, batch, s,
                                    base > 0 ? static_cast<TV *>(ws) : nullptr)));
        return launch_relayout<TV>(xi, static_cast<TV *>(x), op.nn, batch, true, s);
    });
}

// The body of normal_apply once the arguments are checked; ws holds at least
// normal_ws_bytes(op, batch) bytes.
static int normal_apply_into(const Op &op, double alpha, double lambda, double sigma, const void *x,
                             void *out, double *dot_out, int32_t batch, void *ws, hipStream_t s)
{
    return dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        Carver c(ws);
        TV *xT = op.need_T ? c.take<TV>(op.nn * batch) : nullptr;
        TV *y = c.take<TV>(op.rows * batch);
        double *part = c.take<double>(op.n_ag * batch);
        TV *scr = c.take<TV>(prod_scratch_elems(op, batch));
        const TV *xx = static_cast<const TV *>(x);
        if (xT) SCT_TRY(launch_transpose<TV>(op, xx, xT, batch, s));
        SCT_TRY(launch_fwd<TM, TV>(op, xx, xT, y, batch, s, fwd_part_elems(op, batch) ? scr : nullptr));
        SCT_TRY(launch_adj<TM, TV>(op, y, xx, static_cast<TV *>(out), alpha, lambda, sigma,
                                   dot_out ? part : nullptr, batch, s,
                                   adj_scratch_elems(op, batch) ? scr : nullptr));
        if (dot_out) SCT_TRY(launch_sum_partials(part, adj_blocks(op), dot_out, batch, s));
        return RADON_OK;
    });
}

static int check_normal_args(const radon_op *p, const void *x, const void *out, int32_t batch)
{
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    if (!x || !out) return set_error(RADON_EINVAL, "x and out must be non-NULL");
    if (x == out) return set_error(RADON_EINVAL, "out must not alias x");
    return RADON_OK;
}

extern "C" int normal_apply(const radon_op *p, double alpha, double lambda, double sigma,
                            const void *x, void *out, double *dot_out, int32_t batch, int32_t layout,
                            void *ws, int64_t ws_bytes, void *stream)
{
    clear_error();
    SCT_TRY(check_normal_args(p, x, out, batch));
    SCT_TRY(check_layout(layout));
    const Op &op = *as_op(p);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t base = normal_ws_bytes(op, batch);
    if (!relays(layout, batch)) {
        SCT_TRY(check_ws(ws, ws_bytes, base, "normal_apply"));
        return normal_apply_into(op, alpha, lambda, sigma, x, out, dot_out, batch, ws, s);
    }
    SCT_TRY(check_ws(ws, ws_bytes, base + pixel_layout_extra(op, RADON_WS_NORMAL, batch), "normal_apply"));
    return dispatch(op, [&](auto *, auto *tv) {
        using TV = std::remove_pointer_t<decltype(tv)>;
        TV *xi = nullptr, *oi = nullptr;
        relay_buffers<TV>(ws, base, op.nn * batch, op.nn * batch, &xi, &oi);
        SCT_TRY(launch_relayout<TV>(static_cast<const TV *>(x), xi, op.nn, batch, false, s));
        SCT_TRY(normal_apply_into(op, alpha, lambda, sigma, xi, oi, dot_out, batch, ws, s));
        return launch_relayout<TV>(oi, static_cast<TV *>(out), op.nn, batch, true, s);
    });
}

// ---------------------------------------------------------------------------
// normal_apply without a caller workspace: the transposed image, the
// sinogram, the band partials and the <x, out> partials live in a file-scope
// device array instead.  Each device that runs the library holds its own copy
// of the array; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (the array's name in
// host code is a host-side stand-in, not a device address).
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[RADON_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Address of the current device's copy of `scratch` (looked up once per device).
static int scratch_for_current_device(void **out)
{
    int dev = -1;
    SCT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(RADON_EUNSUPPORTED, "device ordinal %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        SCT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return set_error(RADON_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return RADON_OK;
}

extern "C" int normal_apply_noalloc(const radon_op *p, double alpha, double lambda, double sigma,
                                    const void *x, void *out, double *dot_out, int32_t batch,
                                    void *stream)
{
    clear_error();
    SCT_TRY(check_normal_args(p, x, out, batch));
    const Op &op = *as_op(p);
    const int64_t need = normal_ws_bytes(op, batch);
    if (need > RADON_NOALLOC_SCRATCH_BYTES)
        return set_error(RADON_EWORKSPACE,
                         "normal_apply_noalloc: this operator needs %lld bytes of scratch for batch %d, "
                         "beyond the library's fixed %lld; use normal_apply with a workspace",
                         (long long)need, batch, (long long)RADON_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    SCT_TRY(scratch_for_current_device(&ws));
    return normal_apply_into(op, alpha, lambda, sigma, x, out, dot_out, batch, ws,
                             static_cast<hipStream_t>(stream));
}

extern "C" int radon_set_tuning(radon_op *p, const radon_tuning *t)
{
    clear_error();
    SCT_TRY(check_op(p));
    if (!t) return set_error(RADON_EINVAL, "tuning is NULL");
    if (t->fwd_waves != 2 && t->fwd_waves != 4)
        return set_error(RADON_EINVAL, "fwd_waves must be 2 or 4 (got %d)", t->fwd_waves);
    if (t->adj_waves != 0 && t->adj_waves != 1 && t->adj_waves != 2 && t->adj_waves != 4)
        return set_error(RADON_EINVAL, "adj_waves must be 0, 1, 2 or 4 (got %d)", t->adj_waves);
    for (int v : {t->fwd_rhs, t->adj_rhs})
        if (v != 1 && v != 4 && v != 8 && v != 16)
            return set_error(RADON_EINVAL, "fwd_rhs and adj_rhs must be 1, 4, 8 or 16 (got %d)", v);
    if (t->fwd_layout != 0 && t->fwd_layout != 1)
        return set_error(RADON_EINVAL, "fwd_layout must be 0 or 1 (got %d)", t->fwd_layout);
    if (t->adj_layout != 0 && t->adj_layout != 1)
        return set_error(RADON_EINVAL, "adj_layout must be 0 or 1 (got %d)", t->adj_layout);
    if (t->reserved != 0) return set_error(RADON_EINVAL, "reserved must be 0 (got %d)", t->reserved);
    if (t->fwd_lines != 0) {
        bool built = false;
        for (const BandSet &b : as_op(p)->bands) built = built || (b.n_bands > 0 && b.lines == t->fwd_lines);
        if (!built)
            return set_error(RADON_EINVAL,
                             "fwd_lines must be 0, or 16, 32, 64 or 128 on an operator of 256 pixels or more (got %d)",
                             t->fwd_lines);
    }
    as_op(p)->tune = *t;
    return RADON_OK;
}

extern "C" int radon_get_tuning(const radon_op *p, radon_tuning *out)
{
    clear_error();
    SCT_TRY(check_op(p));
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    *out = as_op(p)->tune;
    return RADON_OK;
}
