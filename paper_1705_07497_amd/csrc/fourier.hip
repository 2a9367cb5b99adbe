// Fourier-domain operator of Sections 2 and 3.1 (eq:four_obj, eq:SBFFT,
// eq:fusedop).
//
// The measured projections' 1-D DFTs sample the image's 2-D Fourier transform
// on polar points xi_p (Fourier slice theorem).  The normal operator of the
// Fourier-domain problem, H = Re(F F^*) with (F^* mu)_p = sum_m mu_m
// exp(-i xi_p . m), is evaluated by Greengard-Lee Gaussian gridding on an
// M x M frequency grid:
//
//   F^* ~ B^* F_D^* A,   F ~ A F_D B,   H ~ Re(A F_D (B B^*) F_D^* A)
//
// with A the deconvolution (pi/tau) exp(|m|^2 tau), F_D^* / F_D the unscaled
// DFTs onto and off the grid, B^* the heat-kernel interpolation at the points
// and B the spreading.  eq:fusedop precomputes B B^*: here it is stored as a
// variable-coefficient stencil over the grid (every nonzero of a row lies
// within 2 m_sp - 1 grid points per dimension), in 8 x 8 tiles of grid points
// with the 64 points' coefficients for one offset contiguous, so the product
// streams the coefficients once with full-line loads and reads the grid from
// LDS.  Tiles that no point's window reaches hold no coefficients.
//
// The grid is kept in centred order: grid point s stands for the frequency
// (s - M/2) 2 pi / M.  The resulting (-1)^m factors and the two 1/M^2 of the
// trapezoid rule are folded into the per-mode scale a1 = sqrt(pi/tau)
// exp(m^2 tau) (-1)^m / M applied at zero-padding and at cropping.  The 2-D
// DFTs are a row pass (transforms of whole grid rows in LDS) and two
// four-step column passes; rows that hold no image mode are skipped on the
// way in and not written on the way out.
#include "cg.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

namespace sct {

template <class T>
struct alignas(2 * sizeof(T)) C2 {
    T x, y;
};

// four consecutive stencil coefficients of one grid point: one 16-byte (FP32)
// or two 16-byte (FP64) loads per lane
template <class TM> struct QuadOf;
template <> struct QuadOf<float> { using type = float4; };
template <> struct QuadOf<double> { using type = double4; };
template <class TM> using Quad = typename QuadOf<TM>::type;

// padded stencil width: offsets dx in [0, Dp) with Dp = D rounded up to 4, the
// padding coefficients zero
__host__ __device__ inline int pad4(int d) { return (d + 3) & ~3; }

constexpr int kFouMaxMsp = 12;
constexpr int kFouMaxGrid = 4096;
constexpr int kFftThreads = 256;
constexpr int kFftLdsBudget = 80 * 1024;   // per workgroup, two per CU

__device__ inline int brev(int i, int logM) { return int(__brev(unsigned(i)) >> (32 - logM)); }

// In-place decimation-in-time DFT (radix-2 butterflies, two stages per pass
// over LDS) of `lines` lines of M points held in bit-reversed
// order in buf (line stride `stride`); natural order on return.  sign -1 for
// exp(-2 pi i j k / M) (F_D^*), +1 for its adjoint F_D; tw[k] =
// exp(-2 pi i k / M), k < M/2.
// Stages st and st + 1 run as one sweep: a thread takes the four points
// i0 + {0, 1, 2, 3} hs of a group of 4 hs, applies the stage-st butterflies
// (twiddle W_2hs^k) to both pairs and then the stage-(st + 1) butterflies
// (W_4hs^k and W_4hs^(k + hs)) in registers, so each pair of stages costs one
// pass over LDS and one barrier.  An odd last stage runs alone.
template <class T>
__device__ inline C2<T> cmul(C2<T> c, C2<T> w)
{
    return C2<T>{c.x * w.x - c.y * w.y, c.x * w.y + c.y * w.x};
}

template <class T>
__device__ void lds_fft(C2<T> *buf, int lines, int M, int logM, int stride, const C2<T> *tw, int sign)
{
    const int half = M >> 1, quarter = M >> 2;
    int st0 = 0;
    for (; st0 + 1 < logM; st0 += 2) {
        const int hs = 1 << st0;
        for (int j = threadIdx.x; j < lines * quarter; j += blockDim.x) {
            const int line = j >> (logM - 2);
            const int jj = j & (quarter - 1);
            const int k = jj & (hs - 1);
            const int i0 = ((jj >> st0) << (st0 + 2)) + k;
            C2<T> w1 = tw[k << (logM - 1 - st0)];
            C2<T> w2 = tw[k << (logM - 2 - st0)];
            C2<T> w3 = tw[(k + hs) << (logM - 2 - st0)];
            if (sign > 0) {
                w1.y = -w1.y;
                w2.y = -w2.y;
                w3.y = -w3.y;
            }
            C2<T> *b = buf + line * stride;
            const C2<T> a0 = b[i0], a1 = b[i0 + hs], a2 = b[i0 + 2 * hs], a3 = b[i0 + 3 * hs];
            const C2<T> t1 = cmul(a1, w1), t3 = cmul(a3, w1);
            const C2<T> c0{a0.x + t1.x, a0.y + t1.y}, c1{a0.x - t1.x, a0.y - t1.y};
            const C2<T> c2{a2.x + t3.x, a2.y + t3.y}, c3{a2.x - t3.x, a2.y - t3.y};
            const C2<T> u2 = cmul(c2, w2), u3 = cmul(c3, w3);
            b[i0] = C2<T>{c0.x + u2.x, c0.y + u2.y};
            b[i0 + 2 * hs] = C2<T>{c0.x - u2.x, c0.y - u2.y};
            b[i0 + hs] = C2<T>{c1.x + u3.x, c1.y + u3.y};
            b[i0 + 3 * hs] = C2<T>{c1.x - u3.x, c1.y - u3.y};
        }
        __syncthreads();
    }
    for (int st = st0; st < logM; ++st) {
        const int hs = 1 << st;
        for (int j = threadIdx.x; j < lines * half; j += blockDim.x) {
            const int line = j >> (logM - 1);
            const int jj = j & (half - 1);
            const int k = jj & (hs - 1);
            const int i0 = ((jj >> st) << (st + 1)) + k;
            C2<T> w = tw[k << (logM - 1 - st)];
            if (sign > 0) w.y = -w.y;
            C2<T> *b = buf + line * stride;
            const C2<T> a = b[i0], c = b[i0 + hs];
            const T tx = c.x * w.x - c.y * w.y, ty = c.x * w.y + c.y * w.x;
            b[i0] = C2<T>{a.x + tx, a.y + ty};
            b[i0 + hs] = C2<T>{a.x - tx, a.y - ty};
        }
        __syncthreads();
    }
}

template <class T>
__device__ inline void load_tw(C2<T> *tw_l, const C2<T> *__restrict__ tw, int M)
{
    for (int k = threadIdx.x; k < (M >> 1); k += blockDim.x) tw_l[k] = tw[k];
}

// grid line index i -> image index along that axis, -1 if i holds no mode
__device__ inline int mode_of(int i, int n, int M)
{
    const int h = n >> 1;
    if (i < n - h) return i + h;
    if (i >= M - h) return i - M + h;
    return -1;
}

// Row pass of F_D^* A: image rows -> grid rows (m_y mod M), zero-padded and
// scaled by a1[iy] a1[ix].  Rows without image modes are not written.
template <class T>
__global__ __launch_bounds__(kFftThreads) void k_fou_rows_fwd(const T *__restrict__ x, C2<T> *__restrict__ G,
                                                              const T *__restrict__ a1,
                                                              const C2<T> *__restrict__ tw, int n,
                                                              int M, int logM, int L, int64_t nn,
                                                              int64_t MM)
{
    extern __shared__ char smem[];
    C2<T> *tw_l = reinterpret_cast<C2<T> *>(smem);
    C2<T> *buf = tw_l + (M >> 1);
    const int stride = M + 1;
    const int64_t xo = int64_t(blockIdx.y) * nn, go = int64_t(blockIdx.y) * MM;
    const int iy0 = blockIdx.x * L;
    load_tw(tw_l, tw, M);
    for (int e = threadIdx.x; e < L * M; e += blockDim.x) {
        const int line = e >> logM, i = e & (M - 1);
        const int iy = iy0 + line;
        C2<T> v{T(0), T(0)};
        const int ix = mode_of(i, n, M);
        if (iy < n && ix >= 0) v.x = a1[iy] * a1[ix] * x[xo + int64_t(iy) * n + ix];
        buf[line * stride + brev(i, logM)] = v;
    }
    __syncthreads();
    lds_fft(buf, L, M, logM, stride, tw_l, -1);
    const int h = n >> 1;
    for (int e = threadIdx.x; e < L * M; e += blockDim.x) {
        const int line = e >> logM, i = e & (M - 1);
        const int iy = iy0 + line;
        if (iy >= n) continue;
        const int g = (iy - h) & (M - 1);
        G[go + int64_t(g) * M + i] = buf[line * stride + i];
    }
}

// Column DFTs of length M = M1 M2 in two passes over 16 adjacent columns
// (four-step form): with row n = M2 n1 + n2 and frequency k = k1 + M1 k2,
//   X[k1 + M1 k2] = sum_n2 W_M2^(n2 k2) W_M^(n2 k1) sum_n1 x[M2 n1 + n2] W_M1^(n1 k1).
// Pass 1 (one n2 per workgroup) does the inner M1-point DFTs and the twiddle
// W_M^(n2 k1), in place: it reads and writes the same rows n2 (mod M2).
// Pass 2 (one k1 per workgroup) does the outer M2-point DFTs from rows
// k1 M2 + n2 to rows k1 + M1 k2 of another buffer.  Every load and store is a
// 256-byte row segment.  FWD: rows without image modes are zero on input.
// !FWD: only the rows of image modes are written in pass 2.
constexpr int kColW = 16;
constexpr int kColMaxLen = 64;

template <class T>
__device__ inline C2<T> tw_pow(const C2<T> *__restrict__ tw, int e, int M, int sign)
{
    // exp(sign 2 pi i e / M) for 0 <= e < M from the half table
    C2<T> w = e < (M >> 1) ? tw[e] : C2<T>{-tw[e - (M >> 1)].x, -tw[e - (M >> 1)].y};
    if (sign > 0) w.y = -w.y;
    return w;
}

template <class T, bool FWD, int PASS>
__global__ __launch_bounds__(kFftThreads) void k_fou_cols4(const C2<T> *__restrict__ src,
                                                           C2<T> *__restrict__ dst,
                                                           const C2<T> *__restrict__ tw, int n,
                                                           int M, int logM, int logM1, int logM2,
                                                           int64_t MM)
{
    __shared__ C2<T> buf[kColW * (kColMaxLen + 1)];
    __shared__ C2<T> twl[kColMaxLen / 2];
    const int loglen = PASS == 1 ? logM1 : logM2, len = 1 << loglen;
    const int stride = len + 1;
    const int sel = blockIdx.y;   // n2 in pass 1, k1 in pass 2
    const int c0 = blockIdx.x * kColW;
    const int64_t go = int64_t(blockIdx.z) * MM;
    const int sign = FWD ? -1 : 1;
    for (int k = threadIdx.x; k < (len >> 1); k += blockDim.x) twl[k] = tw[k << (logM - loglen)];
    for (int e = threadIdx.x; e < len * kColW; e += blockDim.x) {
        const int j = e >> 4, col = e & (kColW - 1);
        const int row = PASS == 1 ? (j << logM2) + sel : (sel << logM2) + j;
        C2<T> v{T(0), T(0)};
        if (!(FWD && PASS == 1) || mode_of(row, n, M) >= 0) v = src[go + int64_t(row) * M + c0 + col];
        buf[col * stride + brev(j, loglen)] = v;
    }
    __syncthreads();
    lds_fft(buf, kColW, len, loglen, stride, twl, sign);
    for (int e = threadIdx.x; e < len * kColW; e += blockDim.x) {
        const int k = e >> 4, col = e & (kColW - 1);
        C2<T> v = buf[col * stride + k];
        int row;
        if (PASS == 1) {
            row = (k << logM2) + sel;
            const C2<T> w = tw_pow(tw, (sel * k) & (M - 1), M, sign);
            v = C2<T>{v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x};
        } else {
            row = sel + (k << logM1);
            if (!FWD && mode_of(row, n, M) < 0) continue;
        }
        dst[go + int64_t(row) * M + c0 + col] = v;
    }
}

// Row pass of A F_D with the crop and the normal-operator epilogue:
// h = Re(a1[iy] a1[ix] (F_D v)_m) for the image's modes, then
// out = alpha h + lambda K^T K x + sigma x and one FP64 partial <x, out> per
// workgroup (x may be nullptr when lambda = sigma = 0 and part = nullptr).
template <class T>
__global__ __launch_bounds__(kFftThreads) void k_fou_rows_inv(const C2<T> *__restrict__ G,
                                                              const T *__restrict__ x,
                                                              T *__restrict__ out,
                                                              const T *__restrict__ a1,
                                                              const C2<T> *__restrict__ tw,
                                                              T alpha, T lambda, T sigma,
                                                              double *__restrict__ part, int n,
                                                              int M, int logM, int L, int64_t nn,
                                                              int64_t MM)
{
    extern __shared__ char smem[];
    __shared__ double red[kFftThreads];
    C2<T> *tw_l = reinterpret_cast<C2<T> *>(smem);
    C2<T> *buf = tw_l + (M >> 1);
    const int stride = M + 1;
    const int64_t xo = int64_t(blockIdx.y) * nn, go = int64_t(blockIdx.y) * MM;
    const int iy0 = blockIdx.x * L, h = n >> 1;
    load_tw(tw_l, tw, M);
    for (int e = threadIdx.x; e < L * M; e += blockDim.x) {
        const int line = e >> logM, i = e & (M - 1);
        const int iy = iy0 + line;
        C2<T> v{T(0), T(0)};
        if (iy < n) v = G[go + int64_t((iy - h) & (M - 1)) * M + i];
        buf[line * stride + brev(i, logM)] = v;
    }
    __syncthreads();
    lds_fft(buf, L, M, logM, stride, tw_l, 1);
    double acc = 0.0;
    for (int e = threadIdx.x; e < L * n; e += blockDim.x) {
        const int line = e / n, ix = e - line * n;
        const int iy = iy0 + line;
        if (iy >= n) continue;
        const int i = (ix - h) & (M - 1);
        const T hv = a1[iy] * a1[ix] * buf[line * stride + i].x;
        T o = alpha * hv;
        if (x) {
            const int64_t j = xo + int64_t(iy) * n + ix;
            const T xj = x[j];
            if (lambda != T(0)) {
                T ktk = T(0);   // Neumann 5-point K^T K
                if (ix > 0) ktk += xj - x[j - 1];
                if (ix < n - 1) ktk += xj - x[j + 1];
                if (iy > 0) ktk += xj - x[j - n];
                if (iy < n - 1) ktk += xj - x[j + n];
                o += lambda * ktk;
            }
            if (sigma != T(0)) o += sigma * xj;
            acc += double(xj) * double(o);
        }
        out[xo + int64_t(iy) * n + ix] = o;
    }
    if (!part) return;
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) part[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = tot;
}

// v = (B B^*) u on the grid: 16 x 16 grid points per workgroup (four 8 x 8
// tiles, one wave each); the region plus a periodic halo of R = 2 m_sp - 1
// (one more column for the padded offsets) is staged in LDS, the
// coefficients stream from HBM as quads of offsets (64 lanes x 16 bytes per
// load).  BC images (blockIdx.z selects a chunk of them, nbc present) share
// every coefficient load; with BC = 2 the LDS reads still keep pace with the
// stream.  A tile without coefficients writes zeros.
template <class TM, class T, int BC>
__global__ __launch_bounds__(256) void k_fou_stencil(const C2<T> *__restrict__ u,
                                                     C2<T> *__restrict__ v,
                                                     const Quad<TM> *__restrict__ coef,
                                                     const int32_t *__restrict__ tile_map, int M,
                                                     int R, int64_t MM, int batch)
{
    extern __shared__ char smem[];
    C2<T> *reg = reinterpret_cast<C2<T> *>(smem);
    const int D = 2 * R + 1, Dp = pad4(D), nqx = Dp >> 2;
    const int sh = 16 + 2 * R, sw = 15 + Dp, area = sh * sw;
    const int rx0 = blockIdx.x * 16, ry0 = blockIdx.y * 16;
    const int b0 = blockIdx.z * BC;
    const int nbc = min(BC, batch - b0);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tpr = M >> 3;
    const int blk = tile_map[((ry0 >> 3) + (w >> 1)) * tpr + (rx0 >> 3) + (w & 1)];
    const int any = __syncthreads_or(blk >= 0);
    const int ly = ((w >> 1) << 3) + (lane >> 3), lx = ((w & 1) << 3) + (lane & 7);
    C2<T> acc[BC];
#pragma unroll
    for (int c = 0; c < BC; ++c) acc[c] = C2<T>{T(0), T(0)};
    if (any) {
        for (int c = 0; c < nbc; ++c) {
            const int64_t go = int64_t(b0 + c) * MM;
            for (int e = threadIdx.x; e < area; e += blockDim.x) {
                const int ey = e / sw, ex = e - ey * sw;
                const int gy = (ry0 + ey - R) & (M - 1), gx = (rx0 + ex - R) & (M - 1);
                reg[c * area + e] = u[go + int64_t(gy) * M + gx];
            }
        }
        __syncthreads();
        if (blk >= 0) {
            const Quad<TM> *cq = coef + int64_t(blk) * D * nqx * 64 + lane;
            for (int dy = 0; dy < D; ++dy) {
                const C2<T> *row = reg + (ly + dy) * sw + lx;
                const Quad<TM> *cr = cq + int64_t(dy) * nqx * 64;
#pragma unroll 2
                for (int qx = 0; qx < nqx; ++qx) {
                    const Quad<TM> q = cr[qx * 64];
#pragma unroll
                    for (int c = 0; c < BC; ++c) {
                        if (BC == 1 || c < nbc) {
                            const C2<T> *rc = row + c * area + 4 * qx;
                            const C2<T> u0 = rc[0], u1 = rc[1], u2 = rc[2], u3 = rc[3];
                            acc[c].x += T(q.x) * u0.x + T(q.y) * u1.x + T(q.z) * u2.x + T(q.w) * u3.x;
                            acc[c].y += T(q.x) * u0.y + T(q.y) * u1.y + T(q.z) * u2.y + T(q.w) * u3.y;
                        }
                    }
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < BC; ++c)
        if (BC == 1 || c < nbc) v[int64_t(b0 + c) * MM + int64_t(ry0 + ly) * M + rx0 + lx] = acc[c];
}

// Sum over the 16 lanes of a group (xor tree: a fixed order).
template <class T>
__device__ inline T group16_sum(T v)
{
    for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 16);
    return v;
}

// fhat_p = sum over p's window of G[s] g_p(s) (B^* F_D^* A mu with the
// scales already in G): 16 lanes per point, lane j taking taps j, j + 16, ...
template <class TM, class T>
__global__ __launch_bounds__(256) void k_fou_interp(const C2<T> *__restrict__ G,
                                                    const int32_t *__restrict__ pbase,
                                                    const double *__restrict__ w1d,
                                                    C2<T> *__restrict__ fhat, int64_t P, int M,
                                                    int m_sp, int64_t MM)
{
    const int64_t p = int64_t(blockIdx.x) * 16 + (threadIdx.x >> 4);
    const int j = threadIdx.x & 15;
    const int W = 2 * m_sp;
    const int64_t go = int64_t(blockIdx.y) * MM;
    T ax = T(0), ay = T(0);
    if (p < P) {
        const int y0 = pbase[2 * p] - m_sp + 1, x0 = pbase[2 * p + 1] - m_sp + 1;
        const double *wy = w1d + p * 2 * W, *wx = wy + W;
        for (int t = j; t < W * W; t += 16) {
            const int ky = t / W, kx = t - ky * W;
            const T g = T(TM(wy[ky] * wx[kx]));
            const C2<T> val = G[go + int64_t((y0 + ky) & (M - 1)) * M + ((x0 + kx) & (M - 1))];
            ax += g * val.x;
            ay += g * val.y;
        }
    }
    ax = group16_sum(ax);
    ay = group16_sum(ay);
    if (p < P && j == 0) fhat[int64_t(blockIdx.y) * P + p] = C2<T>{ax, ay};
}

// G[s] = sum_p g_p(s) fhat_p (the spreading B, CSR over grid points): 16
// lanes per grid point; each workgroup takes a run of 16 neighbouring grid
// points, the runs in order of their longest row (rows near the origin hold
// over a thousand entries, the median about 16), so the long rows do not
// form the tail of the launch.
template <class TM, class T>
__global__ __launch_bounds__(256) void k_fou_spread(const C2<T> *__restrict__ fhat,
                                                    const int64_t *__restrict__ sp_ptr,
                                                    const int32_t *__restrict__ sp_pt,
                                                    const TM *__restrict__ sp_w,
                                                    const int32_t *__restrict__ sp_order,
                                                    C2<T> *__restrict__ G, int64_t P, int64_t MM)
{
    const int64_t o = int64_t(blockIdx.x) * 16 + (threadIdx.x >> 4);
    const int j = threadIdx.x & 15;
    const C2<T> *f = fhat + int64_t(blockIdx.y) * P;
    const int64_t s = o < MM ? sp_order[o] : 0;
    T ax = T(0), ay = T(0);
    if (o < MM) {
#pragma unroll 4
        for (int64_t k = sp_ptr[s] + j; k < sp_ptr[s + 1]; k += 16) {
            const T g = T(sp_w[k]);
            const C2<T> val = f[sp_pt[k]];
            ax += g * val.x;
            ay += g * val.y;
        }
    }
    ax = group16_sum(ax);
    ay = group16_sum(ay);
    if (o < MM && j == 0) G[int64_t(blockIdx.y) * MM + s] = C2<T>{ax, ay};
}

// B B^* coefficients of one stored tile and one chunk of 64 padded offsets
// (d' = dy Dp + dx): C[s][d] = sum over points p whose window holds s of
// g_p(s) g_p(s + d), accumulated in FP64 in a fixed order (cells by row,
// points by index) and stored in the matrix value type, in quads of four
// consecutive offsets per grid point.  A point p in cell b (per dimension)
// holds grid points b - m_sp + 1 .. b + m_sp, so the points that reach the
// tile [t0, t0 + 8) sit in cells t0 - m_sp .. t0 + m_sp + 6 (periodic); each
// cell is visited in the unwrapped frame of the tile, where s + d is
// measured.
template <class TM>
__global__ __launch_bounds__(64) void k_fou_build(const int32_t *__restrict__ tiles,
                                                  const int32_t *__restrict__ cell_ptr,
                                                  const int32_t *__restrict__ cell_pts,
                                                  const double *__restrict__ w1d,
                                                  Quad<TM> *__restrict__ coef, int M, int m_sp)
{
    __shared__ double wl[4 * kFouMaxMsp];
    __shared__ int dyx[2][64];
    const int W = 2 * m_sp, R = W - 1, D = 2 * R + 1, Dp = pad4(D), DDp = D * Dp;
    const int blk = blockIdx.x, d0 = blockIdx.y * 64;
    const int tpr = M >> 3;
    const int t = tiles[blk];
    const int t0y = (t / tpr) << 3, t0x = (t % tpr) << 3;
    const int lane = threadIdx.x;
    const int sy = t0y + (lane >> 3), sx = t0x + (lane & 7);
    const int nd = min(64, DDp - d0);   // a multiple of 4
    if (lane < nd) {
        const int d = d0 + lane, dx = d % Dp;
        dyx[0][lane] = d / Dp - R;
        dyx[1][lane] = dx < D ? dx - R : 4 * kFouMaxMsp;   // padding: never inside a window
    }
    double acc[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) acc[j] = 0.0;
    for (int cyu = t0y - m_sp; cyu <= t0y + m_sp + 6; ++cyu) {
        const int cy = cyu & (M - 1);
        const int ky = sy - (cyu - m_sp + 1);
        for (int cxu = t0x - m_sp; cxu <= t0x + m_sp + 6; ++cxu) {
            const int c = cy * M + (cxu & (M - 1));
            const int kx = sx - (cxu - m_sp + 1);
            const int k1 = cell_ptr[c + 1];
            for (int k = cell_ptr[c]; k < k1; ++k) {
                const int64_t p = cell_pts[k];
                __syncthreads();
                if (lane < 2 * W) wl[lane] = w1d[p * 2 * W + lane];
                __syncthreads();
                if (ky < 0 || ky >= W || kx < 0 || kx >= W) continue;
                const double ws = wl[ky] * wl[W + kx];
#pragma unroll
                for (int j = 0; j < 64; ++j) {
                    if (j < nd) {
                        const int ky2 = ky + dyx[0][j], kx2 = kx + dyx[1][j];
                        if (ky2 >= 0 && ky2 < W && kx2 >= 0 && kx2 < W)
                            acc[j] += ws * (wl[ky2] * wl[W + kx2]);
                    }
                }
            }
        }
    }
    Quad<TM> *out = coef + (int64_t(blk) * (DDp >> 2) + (d0 >> 2)) * 64 + lane;
#pragma unroll
    for (int jq = 0; jq < 16; ++jq)
        if (4 * jq < nd) {
            Quad<TM> q;
            q.x = TM(acc[4 * jq]);
            q.y = TM(acc[4 * jq + 1]);
            q.z = TM(acc[4 * jq + 2]);
            q.w = TM(acc[4 * jq + 3]);
            out[int64_t(jq) * 64] = q;
        }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <class T>
static int64_t fft_lds_bytes(int M, int L)
{
    return int64_t(sizeof(C2<T>)) * (int64_t(M / 2) + int64_t(L) * (M + 1));
}

template <class T>
static int fft_lines(int M)
{
    int L = 16;
    while (L > 1 && fft_lds_bytes<T>(M, L) > kFftLdsBudget) L >>= 1;
    return L;
}

static int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

int64_t fourier_parts(const Fou &f) { return (f.n + f.Lr - 1) / f.Lr; }

// two M x M complex grids and the point values, per image
int64_t fourier_grid_bytes(const Fou &f, int batch)
{
    const int64_t g = int64_t(f.vsize) * 2 * int64_t(f.M) * f.M * batch;
    const int64_t pv = int64_t(f.vsize) * 2 * f.P * batch;
    return 2 * ((g + 255) & ~int64_t(255)) + ((pv + 255) & ~int64_t(255));
}

template <class T>
static void split_grids(const Fou &f, void *grids, int batch, C2<T> **g0, C2<T> **g1, C2<T> **fh)
{
    Carver c(grids);
    *g0 = c.take<C2<T>>(int64_t(f.M) * f.M * batch);
    *g1 = c.take<C2<T>>(int64_t(f.M) * f.M * batch);
    *fh = c.take<C2<T>>(f.P * batch);
}

// Column passes of a 2-D DFT: G (in place, pass 1) then G -> out (pass 2).
template <class T, bool FWD>
static int col_passes(const Fou &f, C2<T> *G, C2<T> *out, int batch, hipStream_t s)
{
    const int64_t MM = int64_t(f.M) * f.M;
    const int l1 = (f.logM + 1) / 2, l2 = f.logM - l1;
    const unsigned cb = unsigned(f.M / kColW);
    k_fou_cols4<T, FWD, 1><<<dim3(cb, unsigned(1 << l2), unsigned(batch)), kFftThreads, 0, s>>>(
        G, G, static_cast<const C2<T> *>(f.tw), f.n, f.M, f.logM, l1, l2, MM);
    SCT_TRY(check_launch("k_fou_cols4<1>"));
    k_fou_cols4<T, FWD, 2><<<dim3(cb, unsigned(1 << l1), unsigned(batch)), kFftThreads, 0, s>>>(
        G, out, static_cast<const C2<T> *>(f.tw), f.n, f.M, f.logM, l1, l2, MM);
    return check_launch("k_fou_cols4<2>");
}

// out = F_D^* A x (scaled, centred grid); G is scratch.
template <class T>
static int fwd_to_grid(const Fou &f, const T *x, C2<T> *G, C2<T> *out, int batch, hipStream_t s)
{
    const int64_t MM = int64_t(f.M) * f.M;
    const size_t lr = size_t(fft_lds_bytes<T>(f.M, f.Lr));
    k_fou_rows_fwd<T><<<dim3(unsigned((f.n + f.Lr - 1) / f.Lr), unsigned(batch)), kFftThreads, lr, s>>>(
        x, G, static_cast<const T *>(f.a1), static_cast<const C2<T> *>(f.tw), f.n, f.M, f.logM, f.Lr,
        f.op->nn, MM);
    SCT_TRY(check_launch("k_fou_rows_fwd"));
    return col_passes<T, true>(f, G, out, batch, s);
}

// out = alpha Re(A F_D G) (+ lambda K^T K x + sigma x, partials); G is
// overwritten and S is scratch.
template <class T>
static int grid_to_image(const Fou &f, C2<T> *G, C2<T> *S, const T *x, T *out, double alpha,
                         double lambda, double sigma, double *part, int batch, hipStream_t s)
{
    const int64_t MM = int64_t(f.M) * f.M;
    const size_t lr = size_t(fft_lds_bytes<T>(f.M, f.Lr));
    SCT_TRY((col_passes<T, false>(f, G, S, batch, s)));
    k_fou_rows_inv<T><<<dim3(unsigned(fourier_parts(f)), unsigned(batch)), kFftThreads, lr, s>>>(
        S, x, out, static_cast<const T *>(f.a1), static_cast<const C2<T> *>(f.tw), T(alpha),
        T(lambda), T(sigma), part, f.n, f.M, f.logM, f.Lr, f.op->nn, MM);
    return check_launch("k_fou_rows_inv");
}

template <class TM, class T>
static int interp(const Fou &f, const C2<T> *G, C2<T> *fhat, int batch, hipStream_t s)
{
    k_fou_interp<TM, T><<<dim3(unsigned((f.P + 15) / 16), unsigned(batch)), 256, 0, s>>>(
        G, f.pbase, f.w1d, fhat, f.P, f.M, f.m_sp, int64_t(f.M) * f.M);
    return check_launch("k_fou_interp");
}

template <class TM, class T>
static int spread(const Fou &f, const C2<T> *fhat, C2<T> *G, int batch, hipStream_t s)
{
    const int64_t MM = int64_t(f.M) * f.M;
    k_fou_spread<TM, T><<<dim3(unsigned((MM + 15) / 16), unsigned(batch)), 256, 0, s>>>(
        fhat, f.sp_ptr, f.sp_pt, static_cast<const TM *>(f.sp_w), f.sp_order, G, f.P, MM);
    return check_launch("k_fou_spread");
}

template <class TM, class T>
static int stencil(const Fou &f, const C2<T> *u, C2<T> *v, int batch, hipStream_t s)
{
    const int R = f.D / 2;
    const size_t area = size_t(16 + 2 * R) * size_t(15 + pad4(f.D));
    const unsigned g = unsigned(f.M / 16);
    const int64_t MM = int64_t(f.M) * f.M;
    const Quad<TM> *c = static_cast<const Quad<TM> *>(f.coef);
    if (batch >= 2) {
        k_fou_stencil<TM, T, 2><<<dim3(g, g, unsigned((batch + 1) / 2)), 256, 2 * area * sizeof(C2<T>), s>>>(
            u, v, c, f.tile_map, f.M, R, MM, batch);
    } else {
        k_fou_stencil<TM, T, 1><<<dim3(g, g, 1), 256, area * sizeof(C2<T>), s>>>(
            u, v, c, f.tile_map, f.M, R, MM, batch);
    }
    return check_launch("k_fou_stencil");
}

template <class TM, class TV>
int launch_fourier_normal(const Fou &f, int path, double alpha, double lambda, double sigma,
                          const TV *x, TV *out, double *part, int batch, void *grids, hipStream_t s)
{
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    C2<TV> *g0, *g1, *fh;
    split_grids<TV>(f, grids, batch, &g0, &g1, &fh);
    SCT_TRY(fwd_to_grid<TV>(f, x, g0, g1, batch, s));
    if (path == RADON_FOURIER_FUSED) {
        SCT_TRY((stencil<TM, TV>(f, g1, g0, batch, s)));
    } else {   // F^* to the points, then F back to the grid
        SCT_TRY((interp<TM, TV>(f, g1, fh, batch, s)));
        SCT_TRY((spread<TM, TV>(f, fh, g0, batch, s)));
    }
    return grid_to_image<TV>(f, g0, g1, x, out, alpha, lambda, sigma, part, batch, s);
}

template <class TM, class TV>
int launch_fourier_adj(const Fou &f, const TV *fhat, TV *x, double alpha, int batch, void *grids,
                       hipStream_t s)
{
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    C2<TV> *g0, *g1, *fh;
    split_grids<TV>(f, grids, batch, &g0, &g1, &fh);
    SCT_TRY((spread<TM, TV>(f, reinterpret_cast<const C2<TV> *>(fhat), g0, batch, s)));
    return grid_to_image<TV>(f, g0, g1, nullptr, x, alpha, 0.0, 0.0, nullptr, batch, s);
}

#define SCT_FOU_INST(TM, TV)                                                                       \
    template int launch_fourier_normal<TM, TV>(const Fou &, int, double, double, double,           \
                                               const TV *, TV *, double *, int, void *,            \
                                               hipStream_t);                                       \
    template int launch_fourier_adj<TM, TV>(const Fou &, const TV *, TV *, double, int, void *,    \
                                            hipStream_t);
SCT_FOU_INST(float, float)
SCT_FOU_INST(double, double)
SCT_FOU_INST(float, double)
#undef SCT_FOU_INST

template <class T>
static int set_fft_lds(int64_t bytes)
{
    if (bytes <= 64 * 1024) return RADON_OK;
    for (const void *k : {reinterpret_cast<const void *>(&k_fou_rows_fwd<T>),
                          reinterpret_cast<const void *>(&k_fou_rows_inv<T>)})
        SCT_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
    return RADON_OK;
}

// ---------------------------------------------------------------------------
// construction
// ---------------------------------------------------------------------------

static void free_fou(Fou *f)
{
    if (!f) return;
    for (void *p : f->owned) (void)hipFree(p);
    delete f;
}

static int fou_alloc(Fou &f, void **p, int64_t bytes)
{
    *p = nullptr;
    const hipError_t e = hipMalloc(p, size_t(bytes > 0 ? bytes : 256));
    if (e != hipSuccess)
        return set_error(RADON_EHIP, "hipMalloc of %lld bytes failed: %s", (long long)bytes,
                         hipGetErrorString(e));
    f.owned.push_back(*p);
    f.device_bytes += bytes;
    return RADON_OK;
}

template <class U>
static int fou_upload(Fou &f, U **dst, const std::vector<U> &src)
{
    SCT_TRY(fou_alloc(f, reinterpret_cast<void **>(dst), int64_t(sizeof(U)) * int64_t(src.size())));
    if (!src.empty())
        SCT_HIP(hipMemcpy(*dst, src.data(), sizeof(U) * src.size(), hipMemcpyHostToDevice));
    return RADON_OK;
}

// Points, windows and weights (host, FP64), the gridding CSR, the tile map;
// then B B^* on the device.
template <class TM, class TV>
static int build_fou(Fou &f, hipStream_t st)
{
    const Op &op = *f.op;
    const int M = f.M, W = 2 * f.m_sp;
    const int Q = (op.n_bins - 1) / 2;
    const int nq = 2 * Q + 1;
    f.P = int64_t(op.n_meas) * nq;
    if (f.P * W * W >= (int64_t(1) << 40) || f.P > 0x7fffffff)
        return set_error(RADON_EOVERFLOW, "%lld sample points exceed the gridding tables", (long long)f.P);
    const double h = 2.0 * M_PI / M;
    std::vector<int32_t> pbase(size_t(2 * f.P));
    std::vector<double> w1d(size_t(f.P) * size_t(2 * W));
    for (int a = 0; a < op.n_meas; ++a) {
        const double th = M_PI * op.meas[size_t(a)] / op.n_angles;
        const double ct = std::cos(th), sn = std::sin(th);
        for (int q = -Q; q <= Q; ++q) {
            const int64_t p = int64_t(a) * nq + q + Q;
            const double rho = 2.0 * M_PI * q / op.n_bins;
            const double xi[2] = {sn * rho, ct * rho};   // (y, x)
            for (int dim = 0; dim < 2; ++dim) {
                const int64_t b = int64_t(std::floor(xi[dim] / h));
                pbase[size_t(2 * p + dim)] = int32_t(b + M / 2);
                for (int k = 0; k < W; ++k) {
                    const double l = double(b - f.m_sp + 1 + k);
                    const double dlt = xi[dim] - l * h;
                    w1d[size_t(p * 2 * W + dim * W + k)] = std::exp(-(dlt * dlt) / (4.0 * f.tau));
                }
            }
        }
    }
    // cells (base grid point) -> points, ascending
    const int64_t MM = int64_t(M) * M;
    std::vector<int32_t> cell_ptr(size_t(MM + 1), 0), cell_pts(size_t(f.P));
    for (int64_t p = 0; p < f.P; ++p) ++cell_ptr[size_t(int64_t(pbase[size_t(2 * p)]) * M + pbase[size_t(2 * p + 1)] + 1)];
    for (int64_t c = 0; c < MM; ++c) cell_ptr[size_t(c + 1)] += cell_ptr[size_t(c)];
    {
        std::vector<int32_t> fill(cell_ptr.begin(), cell_ptr.end() - 1);
        for (int64_t p = 0; p < f.P; ++p)
            cell_pts[size_t(fill[size_t(int64_t(pbase[size_t(2 * p)]) * M + pbase[size_t(2 * p + 1)])]++)] = int32_t(p);
    }
    // gridding B as CSR over grid points, points ascending within a row
    f.sp_nnz = f.P * W * W;
    std::vector<int64_t> sp_ptr(size_t(MM + 1), 0);
    auto grid_of = [&](int64_t p, int ky, int kx) {
        const int gy = (pbase[size_t(2 * p)] - f.m_sp + 1 + ky) & (M - 1);
        const int gx = (pbase[size_t(2 * p + 1)] - f.m_sp + 1 + kx) & (M - 1);
        return int64_t(gy) * M + gx;
    };
    for (int64_t p = 0; p < f.P; ++p)
        for (int ky = 0; ky < W; ++ky)
            for (int kx = 0; kx < W; ++kx) ++sp_ptr[size_t(grid_of(p, ky, kx) + 1)];
    for (int64_t c = 0; c < MM; ++c) sp_ptr[size_t(c + 1)] += sp_ptr[size_t(c)];
    std::vector<int32_t> sp_pt(size_t(f.sp_nnz));
    std::vector<TM> sp_w(size_t(f.sp_nnz));
    {
        std::vector<int64_t> fill(sp_ptr.begin(), sp_ptr.end() - 1);
        for (int64_t p = 0; p < f.P; ++p)
            for (int ky = 0; ky < W; ++ky)
                for (int kx = 0; kx < W; ++kx) {
                    const int64_t k = fill[size_t(grid_of(p, ky, kx))]++;
                    sp_pt[size_t(k)] = int32_t(p);
                    sp_w[size_t(k)] = TM(w1d[size_t(p * 2 * W + ky)] * w1d[size_t(p * 2 * W + W + kx)]);
                }
    }
    // grid points for the spreading: runs of 16 consecutive grid points (one
    // workgroup of k_fou_spread), the runs by descending longest row (ties by
    // index), each run in grid order.  Long runs do not form the tail of the
    // launch, and the rows of one workgroup are neighbours, whose entries lie
    // next to each other in sp_pt and sp_w, so no cache line of them is read
    // twice (with the rows one by one by length, a workgroup's 16 rows came
    // from all over the grid).
    std::vector<int32_t> sp_order(static_cast<size_t>(MM));
    {
        const int64_t runs = MM / 16;   // M is a power of two >= 16
        std::vector<int64_t> len(static_cast<size_t>(runs), 0);
        for (int64_t c = 0; c < MM; ++c)
            len[size_t(c / 16)] = std::max(len[size_t(c / 16)], sp_ptr[size_t(c + 1)] - sp_ptr[size_t(c)]);
        std::vector<int64_t> run(static_cast<size_t>(runs));
        for (int64_t r = 0; r < runs; ++r) run[size_t(r)] = r;
        std::stable_sort(run.begin(), run.end(), [&](int64_t a, int64_t c) { return len[size_t(a)] > len[size_t(c)]; });
        for (int64_t i = 0; i < runs; ++i)
            for (int k = 0; k < 16; ++k) sp_order[size_t(i * 16 + k)] = int32_t(run[size_t(i)] * 16 + k);
    }
    // 8 x 8 tiles that some window reaches
    const int tpr = M / 8;
    std::vector<int32_t> tile_map(size_t(tpr) * size_t(tpr), -1);
    for (int64_t p = 0; p < f.P; ++p)
        for (int ky = 0; ky < W; ++ky) {
            const int ty = ((pbase[size_t(2 * p)] - f.m_sp + 1 + ky) & (M - 1)) >> 3;
            for (int kx = 0; kx < W; ++kx) {
                const int tx = ((pbase[size_t(2 * p + 1)] - f.m_sp + 1 + kx) & (M - 1)) >> 3;
                tile_map[size_t(ty * tpr + tx)] = 0;
            }
        }
    std::vector<int32_t> tiles;
    for (int t = 0; t < tpr * tpr; ++t)
        if (tile_map[size_t(t)] == 0) {
            tile_map[size_t(t)] = int32_t(tiles.size());
            tiles.push_back(t);
        }
    f.n_tiles = int64_t(tiles.size());
    // scales and twiddles
    std::vector<TV> a1(size_t(f.n));
    for (int ix = 0; ix < f.n; ++ix) {
        const int m = ix - f.n / 2;
        const double sg = (m & 1) ? -1.0 : 1.0;
        a1[size_t(ix)] = TV(std::sqrt(M_PI / f.tau) * std::exp(double(m) * m * f.tau) * sg / M);
    }
    std::vector<C2<TV>> tw(size_t(M / 2));
    for (int k = 0; k < M / 2; ++k)
        tw[size_t(k)] = C2<TV>{TV(std::cos(2.0 * M_PI * k / M)), TV(-std::sin(2.0 * M_PI * k / M))};

    int32_t *d_cell_ptr = nullptr, *d_cell_pts = nullptr, *d_tiles = nullptr;
    TM *d_spw = nullptr;
    TV *d_a1 = nullptr;
    C2<TV> *d_tw = nullptr;
    SCT_TRY(fou_upload(f, &f.pbase, pbase));
    SCT_TRY(fou_upload(f, &f.w1d, w1d));
    SCT_TRY(fou_upload(f, &f.sp_ptr, sp_ptr));
    SCT_TRY(fou_upload(f, &f.sp_pt, sp_pt));
    SCT_TRY(fou_upload(f, &d_spw, sp_w));
    f.sp_w = d_spw;
    SCT_TRY(fou_upload(f, &f.sp_order, sp_order));
    SCT_TRY(fou_upload(f, &f.tile_map, tile_map));
    SCT_TRY(fou_upload(f, &d_a1, a1));
    f.a1 = d_a1;
    SCT_TRY(fou_upload(f, &d_tw, tw));
    f.tw = d_tw;
    // build-only tables: freed at the end of the build
    Fou tmp;
    SCT_TRY(fou_upload(tmp, &d_cell_ptr, cell_ptr));
    struct Guard {
        Fou &t;
        ~Guard()
        {
            for (void *p : t.owned) (void)hipFree(p);
            t.owned.clear();
        }
    } guard{tmp};
    SCT_TRY(fou_upload(tmp, &d_cell_pts, cell_pts));
    SCT_TRY(fou_upload(tmp, &d_tiles, tiles));
    const int64_t DDp = int64_t(f.D) * pad4(f.D);
    SCT_TRY(fou_alloc(f, &f.coef, int64_t(sizeof(TM)) * f.n_tiles * DDp * 64));
    if (f.n_tiles > 0) {
        if (f.n_tiles > 0x7fffffff) return set_error(RADON_EOVERFLOW, "too many tiles");
        const unsigned chunks = unsigned((DDp + 63) / 64);
        k_fou_build<TM><<<dim3(unsigned(f.n_tiles), chunks), 64, 0, st>>>(
            d_tiles, d_cell_ptr, d_cell_pts, f.w1d, static_cast<Quad<TM> *>(f.coef), M, f.m_sp);
        SCT_TRY(check_launch("k_fou_build"));
    }
    SCT_HIP(hipStreamSynchronize(st));
    SCT_TRY(set_fft_lds<TV>(fft_lds_bytes<TV>(f.M, f.Lr)));
    const int R = f.D / 2;
    const int64_t slds = int64_t(sizeof(C2<TV>)) * (16 + 2 * R) * (15 + pad4(f.D));
    if (slds > 64 * 1024)
        SCT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fou_stencil<TM, TV, 1>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(slds)));
    if (2 * slds > 64 * 1024)
        SCT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fou_stencil<TM, TV, 2>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(2 * slds)));
    return RADON_OK;
}

static const Fou *as_fou(const radon_fourier *p) { return reinterpret_cast<const Fou *>(p); }

static int check_fou(const radon_fourier *p)
{
    if (!p) return set_error(RADON_EINVAL, "Fourier operator is NULL");
    return RADON_OK;
}

}  // namespace sct

using namespace sct;

extern "C" int radon_fourier_create(const radon_op *p, int32_t m_sp, double tau, int32_t grid,
                                    void *stream, radon_fourier **out)
{
    clear_error();
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    *out = nullptr;
    SCT_TRY(check_op(p));
    const Op &op = *as_op(p);
    if (m_sp < 1 || m_sp > kFouMaxMsp)
        return set_error(RADON_EINVAL, "m_sp must be in [1, %d] (got %d)", kFouMaxMsp, m_sp);
    int M = grid;
    if (M == 0) {
        M = 16;
        while (M < 2 * op.n) M *= 2;
    }
    if (M < 16 || (M & (M - 1)) || M < 2 * op.n)
        return set_error(RADON_EINVAL, "grid must be a power of two >= max(16, 2n) (got %d, n = %d)",
                         grid, op.n);
    if (M > kFouMaxGrid)
        return set_error(RADON_EUNSUPPORTED, "grid %d exceeds %d (n <= %d)", M, kFouMaxGrid,
                         kFouMaxGrid / 2);
    if (2 * m_sp > M) return set_error(RADON_EINVAL, "window 2 m_sp = %d exceeds the grid %d", 2 * m_sp, M);
    if (!(tau >= 0.0) || !std::isfinite(tau)) return set_error(RADON_EINVAL, "tau must be >= 0 and finite");
    if (op.n_bins < 1 || op.n_meas < 1) return set_error(RADON_EINVAL, "no measured rays");
    Fou *f = new (std::nothrow) Fou;
    if (!f) return set_error(RADON_EINVAL, "out of host memory");
    f->op = &op;
    f->n = op.n;
    f->M = M;
    f->logM = ilog2(M);
    f->m_sp = m_sp;
    f->D = 4 * m_sp - 1;
    f->tau = tau > 0.0 ? tau : 4.0 * m_sp / (double(M) * M);
    {
        // the deconvolution exp(|m|^2 tau) at the image corner must stay finite
        const double h = double(op.n / 2 + 1);
        if (2.0 * h * h * f->tau > 600.0) {
            delete f;
            return set_error(RADON_EINVAL, "tau %g is too large for n = %d (the deconvolution overflows)",
                             f->tau, op.n);
        }
    }
    f->dtype = op.dtype;
    f->msize = op.msize;
    f->vsize = op.vsize;
    // lines per FFT workgroup: as many as the LDS budget allows, but few enough
    // that a pass has at least 512 workgroups when the image allows it
    {
        const int Lmax = op.vsize == 4 ? fft_lines<float>(M) : fft_lines<double>(M);
        auto lines_for = [&](int count) {
            int L = 1;
            while (2 * L <= Lmax && count / (2 * L) >= 512) L *= 2;
            return L;
        };
        f->Lr = lines_for(op.n);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int rc = dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        return build_fou<TM, TV>(*f, st);
    });
    if (rc != RADON_OK) {
        free_fou(f);
        return rc;
    }
    *out = reinterpret_cast<radon_fourier *>(f);
    return RADON_OK;
}

extern "C" void radon_fourier_destroy(radon_fourier *f) { free_fou(reinterpret_cast<Fou *>(f)); }

extern "C" int radon_fourier_get_info(const radon_fourier *p, radon_fourier_info *out)
{
    clear_error();
    SCT_TRY(check_fou(p));
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    const Fou &f = *as_fou(p);
    out->n_points = f.P;
    out->grid = f.M;
    out->m_sp = f.m_sp;
    out->tau = f.tau;
    out->fused_tiles = f.n_tiles;
    out->fused_bytes = f.n_tiles * int64_t(f.D) * pad4(f.D) * 64 * f.msize;
    out->spread_nnz = f.sp_nnz;
    out->device_bytes = f.device_bytes;
    return RADON_OK;
}

namespace sct {
int64_t sb_ws_bytes(const Op &op, int batch);
}

static int64_t transform_ws(const Fou &f, int batch)
{
    Carver c(nullptr);
    c.take<char>(fourier_grid_bytes(f, batch));
    c.take<double>(fourier_parts(f) * batch);
    return c.used;
}

extern "C" int64_t radon_fourier_workspace_bytes(const radon_fourier *p, int32_t which, int32_t batch)
{
    clear_error();
    if (check_fou(p) != RADON_OK || check_batch(batch) != RADON_OK) return -1;
    const Fou &f = *as_fou(p);
    if (which == RADON_FWS_TRANSFORM) return transform_ws(f, batch);
    if (which == RADON_FWS_SB) {
        Carver c(nullptr);
        c.take<char>(sb_ws_bytes(*f.op, batch));
        c.take<char>(fourier_grid_bytes(f, batch));
        return c.used;
    }
    set_error(RADON_EINVAL, "unknown workspace kind %d", which);
    return -1;
}

extern "C" int fourier_fwd(const radon_fourier *p, const void *mu, void *fhat, int32_t batch, void *ws,
                           int64_t ws_bytes, void *stream)
{
    clear_error();
    SCT_TRY(check_fou(p));
    SCT_TRY(check_batch(batch));
    if (!mu || !fhat) return set_error(RADON_EINVAL, "mu and fhat must be non-NULL");
    const Fou &f = *as_fou(p);
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    SCT_TRY(check_ws(ws, ws_bytes, transform_ws(f, batch), "fourier_fwd"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    return dispatch(*f.op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        C2<TV> *g0, *g1, *fh;
        split_grids<TV>(f, ws, batch, &g0, &g1, &fh);
        SCT_TRY(fwd_to_grid<TV>(f, static_cast<const TV *>(mu), g0, g1, batch, s));
        return interp<TM, TV>(f, g1, static_cast<C2<TV> *>(fhat), batch, s);
    });
}

extern "C" int fourier_adj(const radon_fourier *p, const void *fhat, void *x, double alpha,
                           int32_t batch, void *ws, int64_t ws_bytes, void *stream)
{
    clear_error();
    SCT_TRY(check_fou(p));
    SCT_TRY(check_batch(batch));
    if (!fhat || !x) return set_error(RADON_EINVAL, "fhat and x must be non-NULL");
    const Fou &f = *as_fou(p);
    SCT_TRY(check_ws(ws, ws_bytes, transform_ws(f, batch), "fourier_adj"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    return dispatch(*f.op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        return launch_fourier_adj<TM, TV>(f, static_cast<const TV *>(fhat), static_cast<TV *>(x), alpha,
                                          batch, ws, s);
    });
}

extern "C" int fourier_normal(const radon_fourier *p, int32_t path, double alpha, double lambda,
                              double sigma, const void *x, void *out, double *dot_out, int32_t batch,
                              void *ws, int64_t ws_bytes, void *stream)
{
    clear_error();
    SCT_TRY(check_fou(p));
    SCT_TRY(check_batch(batch));
    if (path != RADON_FOURIER_FUSED && path != RADON_FOURIER_NUFFT)
        return set_error(RADON_EINVAL, "unknown path %d", path);
    if (!x || !out) return set_error(RADON_EINVAL, "x and out must be non-NULL");
    if (x == out) return set_error(RADON_EINVAL, "out must not alias x");
    const Fou &f = *as_fou(p);
    SCT_TRY(check_ws(ws, ws_bytes, transform_ws(f, batch), "fourier_normal"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver c(ws);
    void *grids = c.take<char>(fourier_grid_bytes(f, batch));
    double *part = c.take<double>(fourier_parts(f) * batch);
    return dispatch(*f.op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        SCT_TRY((launch_fourier_normal<TM, TV>(f, path, alpha, lambda, sigma, static_cast<const TV *>(x),
                                               static_cast<TV *>(out), dot_out ? part : nullptr, batch,
                                               grids, s)));
        if (dot_out) SCT_TRY(launch_sum_partials(part, fourier_parts(f), dot_out, batch, s));
        return RADON_OK;
    });
}
