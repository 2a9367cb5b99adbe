// Conjugate gradients on the normal operator (Section 2: eq:KKT, eq:PD_resolve
// and eq:SB_solve have no closed-form solution and are solved iteratively)
// and anisotropic-TV split Bregman (Goldstein-Osher, the solver of Section 4,
// with inexact inner solves as in Section 3.2).
//
// Vectors stay in the operator dtype; the CG scalars rho, gamma, alpha_k and
// beta_k live in FP64 on the device and are updated by single-block kernels,
// so nothing is read back to the host inside a solve.  Every reduction sums
// FP64 partials in a fixed order, which makes runs bitwise reproducible.
#include "cg.hpp"

#include <functional>

#include <cmath>

namespace sct {

struct SbScal {
    double first, upd_b, upd_u;
    int32_t outer, stop, breakdowns, pad;
};

// ---------------------------------------------------------------------------
// CG kernels
// ---------------------------------------------------------------------------

// p = r (and its transposed copy pT when requested), uprev = u when requested,
// partial <r, r> per 32x32 tile.
template <class T>
__global__ __launch_bounds__(256) void k_cg_start(const T *__restrict__ r, T *__restrict__ p,
                                                  T *__restrict__ pT, const T *__restrict__ u,
                                                  T *__restrict__ uprev, double *__restrict__ part,
                                                  int n, int64_t nn)
{
    __shared__ T tile[32][33];
    __shared__ double red[256];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int64_t off = int64_t(blockIdx.z) * nn;
    double acc = 0.0;
    for (int i = threadIdx.y; i < 32; i += 8) {
        const int iy = by + i, ix = bx + threadIdx.x;
        if (iy < n && ix < n) {
            const int64_t j = off + int64_t(iy) * n + ix;
            const T v = r[j];
            p[j] = v;
            tile[i][threadIdx.x] = v;
            acc += double(v) * double(v);
            if (uprev) uprev[j] = u[j];
        }
    }
    const double tot = block_sum(acc, red);
    if (pT) {
        for (int i = threadIdx.y; i < 32; i += 8) {
            const int ix = bx + i, iy = by + threadIdx.x;
            if (ix < n && iy < n) pT[off + int64_t(ix) * n + iy] = tile[threadIdx.x][i];
        }
    }
    if (threadIdx.x == 0 && threadIdx.y == 0)
        part[int64_t(blockIdx.z) * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = tot;
}

// rho_0 = sum of partials; resets the per-solve state (ring slot 0).  A set
// SB stop flag starts the solve stopped (the outer loop has finished).
__global__ __launch_bounds__(256) void k_cg_begin(const double *__restrict__ part, int64_t count,
                                                  CgState *__restrict__ st,
                                                  const SbScal *__restrict__ sbs)
{
    __shared__ double red[256];
    const int b = blockIdx.x;
    const double rho = sum_part_block(part + int64_t(b) * count, count, red);
    if (threadIdx.x == 0) {
        CgState c;
        c.rho = rho;
        c.rho0 = rho;
        c.stopped = (sbs && sbs[b].stop) ? 1 : 0;
        c.iters = 0;
        c.breakdown = 0;
        c.pad = 0;
        st[b] = c;
    }
}

// Step length and update: gamma = <p, Ap> from the adjoint's partials (every
// block sums them in the same fixed order); stop on rho == 0, on the relative
// tolerance, or on a breakdown (gamma <= 0 or non-finite); otherwise
// a = rho / gamma, x += a p, r -= a q and partial <r, r>.  Block 0 records the
// decision in `step` for the p update.
// FULL: every thread's kPre elements lie in range, so the loads and stores
// carry no per-element test.  (A branch around each store would make the next
// store wait until the previous one has completed.)
template <class T, bool FULL>
__device__ __forceinline__ void cg_xr_body(T *__restrict__ x, T *__restrict__ r,
                                           const T *__restrict__ p, const T *__restrict__ q,
                                           const double *__restrict__ part_adj, int64_t n_adj,
                                           const CgState *__restrict__ st, CgStep *__restrict__ step,
                                           double rtol, double *__restrict__ part, int64_t nn,
                                           double *red)
{
    const int64_t b = blockIdx.y;
    const int64_t off = b * nn;
    const int64_t i0 = int64_t(blockIdx.x) * kVecThreads + threadIdx.x;
    const int64_t stride = int64_t(gridDim.x) * kVecThreads;
    // the first kPre elements' operands are loaded before the step length is
    // known, so their latency overlaps the reduction of the partials
    constexpr int kPre = 4;
    T px[kPre] = {}, pp[kPre] = {}, pq[kPre] = {}, pr[kPre] = {};
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
        const int64_t i = i0 + k * stride;
        if (FULL || i < nn) {
            const int64_t j = off + i;
            if (x) {
                px[k] = x[j];
                pp[k] = p[j];
            }
            pq[k] = q[j];
            pr[k] = r[j];
        }
    }
    const double gamma = sum_part_block(part_adj + b * n_adj, n_adj, red);
    double a;
    const int stop = cg_decide(st[b], gamma, rtol, &a);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        CgStep o;
        o.a = a;
        o.gamma = gamma;
        o.stopped = stop;
        o.pad = 0;
        step[b] = o;
    }
    if (stop) return;   // uniform per block; the partials are then unused
    const T at = T(a);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
        const int64_t i = i0 + k * stride;
        if (FULL || i < nn) {
            const int64_t j = off + i;
            if (x) x[j] = fma(at, pp[k], px[k]);   // a replay only needs r
            const T rn = fma(-at, pq[k], pr[k]);
            r[j] = rn;
            acc += double(rn) * double(rn);
        }
    }
    for (int64_t i = i0 + kPre * stride; i < nn; i += stride) {
        const int64_t j = off + i;
        if (x) x[j] = fma(at, p[j], x[j]);
        const T rn = fma(-at, q[j], r[j]);
        r[j] = rn;
        acc += double(rn) * double(rn);
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) part[b * gridDim.x + blockIdx.x] = tot;
}

template <class T>
__global__ __launch_bounds__(kVecThreads) void k_cg_xr(
    T *__restrict__ x, T *__restrict__ r, const T *__restrict__ p, const T *__restrict__ q,
    const double *__restrict__ part_adj, int64_t n_adj, const CgState *__restrict__ st,
    CgStep *__restrict__ step, double rtol, double *__restrict__ part, int64_t nn)
{
    __shared__ double red[kVecThreads];
    const int64_t stride = int64_t(gridDim.x) * kVecThreads;
    const bool full = int64_t(blockIdx.x) * kVecThreads + (kVecThreads - 1) + 3 * stride < nn;
    if (full)
        cg_xr_body<T, true>(x, r, p, q, part_adj, n_adj, st, step, rtol, part, nn, red);
    else
        cg_xr_body<T, false>(x, r, p, q, part_adj, n_adj, st, step, rtol, part, nn, red);
}

// beta = rho'/rho from the update's partials (summed by every block in the
// same order), p = r + beta p with its transposed copy; block 0 writes the
// next iteration's state.
// FULL: the 32 x 32 tile lies inside the image, so the loads and stores carry
// no per-element test (see cg_xr_body).
template <class T, bool FULL>
__device__ __forceinline__ void cg_p_body(const T *__restrict__ r, T *__restrict__ p,
                                          T *__restrict__ pT, const double *__restrict__ part,
                                          int64_t n_part, const CgState &c,
                                          CgState *__restrict__ st_next, bool lead, int n,
                                          int64_t nn, T (*tile)[33], double *red)
{
    const int64_t b = blockIdx.z;
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int64_t off = b * nn;
    // the tile's r and p are loaded before beta is known (the reduction of
    // the partials overlaps their latency)
    T rr[4] = {}, pp[4] = {};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int iy = by + threadIdx.y + 8 * k, ix = bx + threadIdx.x;
        if (FULL || (iy < n && ix < n)) {
            const int64_t j = off + int64_t(iy) * n + ix;
            rr[k] = r[j];
            pp[k] = p[j];
        }
    }
    double v = 0.0;
    const int t = threadIdx.y * 32 + threadIdx.x;
    for (int64_t i = t; i < n_part; i += 256) v += part[b * n_part + i];
    const double rn = block_sum(v, red);
    const double beta_d = rn / c.rho;
    if (lead) {
        CgState o = c;
        o.rho = rn;
        o.iters = c.iters + 1;
        st_next[b] = o;
    }
    const T beta = T(beta_d);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = threadIdx.y + 8 * k;
        const int iy = by + i, ix = bx + threadIdx.x;
        if (FULL || (iy < n && ix < n)) {
            const T v2 = fma(beta, pp[k], rr[k]);
            p[off + int64_t(iy) * n + ix] = v2;
            tile[i][threadIdx.x] = v2;
        }
    }
    if (!pT) return;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = threadIdx.y + 8 * k;
        const int ix = bx + i, iy = by + threadIdx.x;
        if (FULL || (ix < n && iy < n)) pT[off + int64_t(ix) * n + iy] = tile[threadIdx.x][i];
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_cg_p(const T *__restrict__ r, T *__restrict__ p,
                                              T *__restrict__ pT, const double *__restrict__ part,
                                              int64_t n_part, const CgState *__restrict__ st,
                                              const CgStep *__restrict__ step,
                                              CgState *__restrict__ st_next, int it, int n,
                                              int64_t nn)
{
    __shared__ T tile[32][33];
    __shared__ double red[256];
    const int64_t b = blockIdx.z;
    const CgState c = st[b];
    const int stop = step[b].stopped;
    const bool lead = blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && threadIdx.y == 0;
    if (stop) {
        if (lead) {
            CgState o = c;
            o.stopped = 1;
            if (stop == 2 && !c.stopped) o.breakdown = it + 1;
            st_next[b] = o;
        }
        return;
    }
    const bool full = int(blockIdx.x) * 32 + 32 <= n && int(blockIdx.y) * 32 + 32 <= n;
    if (full)
        cg_p_body<T, true>(r, p, pT, part, n_part, c, st_next, lead, n, nn, tile, red);
    else
        cg_p_body<T, false>(r, p, pT, part, n_part, c, st_next, lead, n, nn, tile, red);
}

__global__ void k_cg_info(const CgState *__restrict__ st, radon_cg_info *__restrict__ info, int batch)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    radon_cg_info o;
    o.iterations = st[b].iters;
    o.breakdown = st[b].breakdown;
    o.rho0 = st[b].rho0;
    o.rho = st[b].rho;
    info[b] = o;
}

// r = a - b (a may alias r)
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_sub(const T *a, const T *__restrict__ b, T *r,
                                                      int64_t count)
{
    for (int64_t i = int64_t(blockIdx.x) * kVecThreads + threadIdx.x; i < count;
         i += int64_t(gridDim.x) * kVecThreads)
        r[i] = a[i] - b[i];
}

// ---------------------------------------------------------------------------
// split Bregman kernels
// ---------------------------------------------------------------------------

template <class T>
__device__ inline T shrink(T z, T g)
{
    const T a = fabs(z) - g;
    if (a <= T(0)) return T(0);
    return z > T(0) ? a : -a;
}

// g = K u; d = shrink(g + b, 1/lambda); b += g - d; dw = (d - b) - (d_old - b_old);
// partials of ||b_new - b_old||_1 and ||u - u_prev||_1.
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_sb_shrink(
    const T *__restrict__ u, const T *__restrict__ uprev, T *__restrict__ dx, T *__restrict__ dy,
    T *__restrict__ bx, T *__restrict__ by, T *__restrict__ dwx, T *__restrict__ dwy, T thresh,
    const SbScal *__restrict__ sbs, double *__restrict__ part, int n, int64_t nn)
{
    __shared__ double red[kVecThreads];
    const int64_t b = blockIdx.y;
    if (sbs[b].stop) return;
    const int64_t off = b * nn;
    double sb_acc = 0.0, su_acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kVecThreads + threadIdx.x; i < nn;
         i += int64_t(gridDim.x) * kVecThreads) {
        const int iy = int(i / n), ix = int(i % n);
        const int64_t j = off + i;
        const T uj = u[j];
        const T gx = ix < n - 1 ? u[j + 1] - uj : T(0);
        const T gy = iy < n - 1 ? u[j + n] - uj : T(0);
        const T obx = bx[j], oby = by[j], odx = dx[j], ody = dy[j];
        const T ndx = shrink(gx + obx, thresh);
        const T ndy = shrink(gy + oby, thresh);
        const T nbx = obx + gx - ndx;
        const T nby = oby + gy - ndy;
        sb_acc += double(fabs(nbx - obx)) + double(fabs(nby - oby));
        su_acc += double(fabs(uj - uprev[j]));
        dwx[j] = (ndx - nbx) - (odx - obx);
        dwy[j] = (ndy - nby) - (ody - oby);
        dx[j] = ndx;
        dy[j] = ndy;
        bx[j] = nbx;
        by[j] = nby;
    }
    const double t1 = block_sum(sb_acc, red);
    const double t2 = block_sum(su_acc, red);
    if (threadIdx.x == 0) {
        part[(b * gridDim.x + blockIdx.x) * 2 + 0] = t1;
        part[(b * gridDim.x + blockIdx.x) * 2 + 1] = t2;
    }
}

// r += lambda K^T dw  (the right-hand side of the next solve grows by
// lambda K^T (w_new - w_old), w = d - b)
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_sb_carry(T *__restrict__ r,
                                                           const T *__restrict__ dwx,
                                                           const T *__restrict__ dwy, T lambda,
                                                           const SbScal *__restrict__ sbs, int n,
                                                           int64_t nn)
{
    const int64_t b = blockIdx.y;
    if (sbs[b].stop) return;
    const int64_t off = b * nn;
    for (int64_t i = int64_t(blockIdx.x) * kVecThreads + threadIdx.x; i < nn;
         i += int64_t(gridDim.x) * kVecThreads) {
        const int iy = int(i / n), ix = int(i % n);
        const int64_t j = off + i;
        T kt = T(0);
        if (ix >= 1) kt += dwx[j - 1];
        if (ix <= n - 2) kt -= dwx[j];
        if (iy >= 1) kt += dwy[j - n];
        if (iy <= n - 2) kt -= dwy[j];
        r[j] += lambda * kt;
    }
}

__global__ __launch_bounds__(256) void k_sb_update(const double *__restrict__ part, int64_t count,
                                                   SbScal *__restrict__ sbs,
                                                   const CgState *__restrict__ sc, double tol)
{
    __shared__ double red[256];
    const int b = blockIdx.x;
    double v1 = 0.0, v2 = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256) {
        v1 += part[(int64_t(b) * count + i) * 2 + 0];
        v2 += part[(int64_t(b) * count + i) * 2 + 1];
    }
    const double ub = block_sum(v1, red);
    const double uu = block_sum(v2, red);
    if (threadIdx.x == 0) {
        SbScal s = sbs[b];
        if (!s.stop) {
            s.outer += 1;
            if (sc[b].breakdown) s.breakdowns += 1;
            if (s.outer == 1) s.first = ub;
            s.upd_b = ub;
            s.upd_u = uu;
            if (tol > 0.0 && s.outer > 1 && ub < tol * s.first) s.stop = 1;
        }
        sbs[b] = s;
    }
}

__global__ void k_sb_reset(SbScal *__restrict__ sbs, int batch)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    SbScal s;
    s.first = 0.0;
    s.upd_b = 0.0;
    s.upd_u = 0.0;
    s.outer = 0;
    s.stop = 0;
    s.breakdowns = 0;
    s.pad = 0;
    sbs[b] = s;
}

__global__ void k_sb_info(const SbScal *__restrict__ sbs, radon_sb_info *__restrict__ info, int batch)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    radon_sb_info o;
    o.outer = sbs[b].outer;
    o.breakdowns = sbs[b].breakdowns;
    o.upd_b_first = sbs[b].first;
    o.upd_b = sbs[b].upd_b;
    o.upd_u = sbs[b].upd_u;
    info[b] = o;
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------

template <class T>
struct CgBufs {
    T *r = nullptr, *p = nullptr, *pT = nullptr, *q = nullptr, *y = nullptr;
    double *part_adj = nullptr, *part_vec = nullptr;
    CgState *st = nullptr;   // [2][batch]
    CgStep *step = nullptr;  // [2][batch]
};

template <class T>
static void carve_cg(const Op &op, int batch, Carver &c, CgBufs<T> &w)
{
    const int64_t nb = op.nn * batch;
    w.r = c.take<T>(nb);
    w.p = c.take<T>(nb);
    w.pT = op.need_T ? c.take<T>(nb) : nullptr;
    w.q = c.take<T>(nb);
    // the products' scratch (band partials, pixel-major copies) follows y
    w.y = c.take<T>(op.rows * batch + prod_scratch_elems(op, batch));
    // one partial per adjoint workgroup, or per image row (the Fourier-domain
    // operator's row pass)
    w.part_adj = c.take<double>((op.n_ag > op.n ? op.n_ag : int64_t(op.n)) * batch);
    const int64_t tl = int64_t(tiles_of(op.n)) * tiles_of(op.n);
    const int64_t pv = tl > 2 * vec_blocks(op.nn) ? tl : 2 * vec_blocks(op.nn);
    w.part_vec = c.take<double>(pv * batch);
    w.st = c.take<CgState>(2 * int64_t(batch));
    w.step = c.take<CgStep>(2 * int64_t(batch));
}

int64_t cg_ws_bytes(const Op &op, int batch)
{
    Carver c(nullptr);
    if (op.vsize == 4) {
        CgBufs<float> w;
        carve_cg(op, batch, c, w);
    } else {
        CgBufs<double> w;
        carve_cg(op, batch, c, w);
    }
    return c.used;
}

template <class T>
struct SbBufs {
    T *dx, *dy, *bx, *by, *dwx, *dwy, *uprev;
    SbScal *sbs;
    double *part;
    CgBufs<T> cg;
};

template <class T>
static void carve_sb(const Op &op, int batch, Carver &c, SbBufs<T> &w)
{
    const int64_t nb = op.nn * batch;
    // persistent state first so that a resumed call finds it at the same place
    w.dx = c.take<T>(nb);
    w.dy = c.take<T>(nb);
    w.bx = c.take<T>(nb);
    w.by = c.take<T>(nb);
    carve_cg(op, batch, c, w.cg);   // cg.r is the carried residual
    w.dwx = c.take<T>(nb);
    w.dwy = c.take<T>(nb);
    w.uprev = c.take<T>(nb);
    w.sbs = c.take<SbScal>(batch);
    w.part = c.take<double>(int64_t(2) * vec_blocks(op.nn) * batch);
}

int64_t sb_ws_bytes(const Op &op, int batch)
{
    Carver c(nullptr);
    if (op.vsize == 4) {
        SbBufs<float> w;
        carve_sb(op, batch, c, w);
    } else {
        SbBufs<double> w;
        carve_sb(op, batch, c, w);
    }
    return c.used;
}

// The operator A of a CG solve.  ExactA is the normal operator of Section 2
// through the stored matrices (forward product into y, then the adjoint with
// the fused epilogue); SurA is the surrogate of Section 3.2 (a stencil, no
// transposed copy needed).  Both leave one FP64 partial of <p, A p> per block
// in part, n_part() of them per right-hand side.
template <class TM, class T>
struct ExactA {
    const Op &op;
    double alpha, lambda, sigma;
    int64_t n_part() const { return adj_blocks(op); }
    bool needs_T() const { return op.need_T; }
    int operator()(const T *p, const T *pT, T *q, T *y, double *part, int batch,
                   hipStream_t s) const
    {
        // y comes from carve_cg, with room for the products' scratch after it
        T *scr = y + op.rows * batch;
        SCT_TRY((launch_fwd<TM, T>(op, p, pT, y, batch, s, fwd_part_elems(op, batch) ? scr : nullptr)));
        return launch_adj<TM, T>(op, y, p, q, alpha, lambda, sigma, part, batch, s,
                                 adj_scratch_elems(op, batch) ? scr : nullptr);
    }
};

template <class T>
struct SurA {
    const Sur &sur;
    double alpha, lambda, sigma;
    int64_t n_part() const { return surrogate_parts(sur); }
    bool needs_T() const { return false; }
    int operator()(const T *p, const T *, T *q, T *, double *part, int batch, hipStream_t s) const
    {
        return launch_surrogate<T>(sur, alpha, lambda, sigma, p, q, part, batch, s);
    }
};

// H of the Fourier-domain problem (eq:SBFFT) by gridding, fused (eq:fusedop)
// or through the two transforms; grids is its scratch.
template <class TM, class T>
struct FouA {
    const Fou &fou;
    int path;
    double alpha, lambda, sigma;
    void *grids;
    int64_t n_part() const { return fourier_parts(fou); }
    bool needs_T() const { return false; }
    int operator()(const T *p, const T *, T *q, T *, double *part, int batch, hipStream_t s) const
    {
        return launch_fourier_normal<TM, T>(fou, path, alpha, lambda, sigma, p, q, part, batch, grids, s);
    }
};

// CG start: p = r (+ transposed copy), rho_0, state in ring slot 0.
template <class T>
static int cg_start(const Op &op, int batch, CgBufs<T> &w, T *u_for_prev, T *uprev,
                    const SbScal *sbs, hipStream_t s)
{
    const unsigned t = unsigned(tiles_of(op.n));
    const dim3 tg{t, t, unsigned(batch)}, tb{32, 8, 1};
    const int64_t ntiles = int64_t(t) * t;
    k_cg_start<T><<<tg, tb, 0, s>>>(w.r, w.p, w.pT, u_for_prev, uprev, w.part_vec, op.n, op.nn);
    SCT_TRY(check_launch("k_cg_start"));
    k_cg_begin<<<unsigned(batch), 256, 0, s>>>(w.part_vec, ntiles, w.st, sbs);
    return check_launch("k_cg_begin");
}

// CG iteration `it`: q = A p, step length, x/r update, p update; state moves
// from ring slot it % 2 to (it + 1) % 2.
template <class T, class AOp>
static int cg_iter(const Op &op, const AOp &A, T *x, int batch, int it, double rtol, CgBufs<T> &w,
                   hipStream_t s, T *rec_q = nullptr, T *rec_p = nullptr, T *rec_r = nullptr)
{
    const unsigned t = unsigned(tiles_of(op.n));
    const dim3 tg{t, t, unsigned(batch)}, tb{32, 8, 1};
    const int vb = vec_blocks(op.nn);
    const int64_t cnt = op.nn * batch;
    const int vbc = vec_blocks(cnt);
    CgState *cur = w.st + int64_t(it & 1) * batch, *nxt = w.st + int64_t((it + 1) & 1) * batch;
    CgStep *stp = w.step + int64_t(it & 1) * batch;
    SCT_TRY(A(w.p, w.pT, w.q, w.y, w.part_adj, batch, s));
    if (rec_q) k_copy<T><<<vbc, kVecThreads, 0, s>>>(w.q, rec_q, cnt);
    if (rec_p) k_copy<T><<<vbc, kVecThreads, 0, s>>>(w.p, rec_p, cnt);
    k_cg_xr<T><<<dim3(unsigned(vb), unsigned(batch)), kVecThreads, 0, s>>>(
        x, w.r, w.p, w.q, w.part_adj, A.n_part(), cur, stp, rtol, w.part_vec, op.nn);
    SCT_TRY(check_launch("k_cg_xr"));
    if (rec_r) k_copy<T><<<vbc, kVecThreads, 0, s>>>(w.r, rec_r, cnt);
    k_cg_p<T><<<tg, tb, 0, s>>>(w.r, w.p, w.pT, w.part_vec, vb, cur, stp, nxt, it, op.n, op.nn);
    return check_launch("k_cg_p");
}

// One CG solve on A(alpha, lambda, sigma) from x with the residual already in
// w.r; the final state is left in ring slot n_iter % 2.
template <class T, class AOp>
static int cg_run(const Op &op, const AOp &A, T *x, int batch, int n_iter, double rtol,
                  CgBufs<T> &w, T *u_for_prev, T *uprev, const SbScal *sbs, hipStream_t s)
{
    SCT_TRY(cg_start<T>(op, batch, w, u_for_prev, uprev, sbs, s));
    for (int it = 0; it < n_iter; ++it) SCT_TRY((cg_iter<T>(op, A, x, batch, it, rtol, w, s)));
    return RADON_OK;
}

static const CgState *final_state(const CgState *st, int n_iter, int batch)
{
    return st + int64_t(n_iter & 1) * batch;
}

// w.q = A x (uses w.pT and w.y as temporaries)
template <class T, class AOp>
static int apply_A_into_q(const Op &op, const AOp &A, const T *x, int batch, CgBufs<T> &w,
                          hipStream_t s)
{
    if (w.pT && A.needs_T()) SCT_TRY(launch_transpose<T>(op, x, w.pT, batch, s));
    return A(x, w.pT, w.q, w.y, nullptr, batch, s);
}

template <class TM, class T>
static int cg_typed(const Op &op, double alpha, double lambda, double sigma, const void *rhs_v,
                    void *x_v, int x0_given, int batch, int n_iter, double rtol, void *ws,
                    radon_cg_info *info, hipStream_t s)
{
    Carver c(ws);
    CgBufs<T> w;
    carve_cg(op, batch, c, w);
    const T *rhs = static_cast<const T *>(rhs_v);
    T *x = static_cast<T *>(x_v);
    const int64_t cnt = op.nn * batch;
    const int vb = vec_blocks(cnt);
    if (x0_given) {
        SCT_TRY((apply_A_into_q<T>(op, ExactA<TM, T>{op, alpha, lambda, sigma}, x, batch, w, s)));
        k_sub<T><<<vb, kVecThreads, 0, s>>>(rhs, w.q, w.r, cnt);
        SCT_TRY(check_launch("k_sub"));
    } else {
        k_fill<T><<<vb, kVecThreads, 0, s>>>(x, T(0), cnt);
        SCT_TRY(check_launch("k_fill"));
        k_copy<T><<<vb, kVecThreads, 0, s>>>(rhs, w.r, cnt);
        SCT_TRY(check_launch("k_copy"));
    }
    SCT_TRY((cg_run<T>(op, ExactA<TM, T>{op, alpha, lambda, sigma}, x, batch, n_iter, rtol, w,
                       nullptr, nullptr, nullptr, s)));
    if (info) {
        k_cg_info<<<unsigned((batch + 63) / 64), 64, 0, s>>>(final_state(w.st, n_iter, batch), info,
                                                             batch);
        SCT_TRY(check_launch("k_cg_info"));
    }
    return RADON_OK;
}

// Split Bregman with the inner CG on A (exact, surrogate or Fourier-domain);
// data_rhs(r) writes the data term of the right-hand side: alpha (MR)^T f
// through the stored adjoint for the sinogram problems (eq:SB_solve,
// eq:surr_SBupd), alpha Re(F fhat) for the Fourier-domain one (eq:SBFFT).
template <class T, class AOp, class RhsF>
static int sb_run(const Op &op, const AOp &A, const RhsF &data_rhs, const radon_sb_params &P,
                  void *mu_v, int batch, void *ws, radon_sb_info *info, hipStream_t s)
{
    Carver c(ws);
    SbBufs<T> w;
    carve_sb(op, batch, c, w);
    if (!A.needs_T()) w.cg.pT = nullptr;   // no transposed direction to keep
    T *u = static_cast<T *>(mu_v);
    const int64_t cnt = op.nn * batch;
    const int vbc = vec_blocks(cnt);
    const int vb = vec_blocks(op.nn);
    const double lambda = P.lambda;
    if (!(P.flags & RADON_SB_RESUME)) {
        for (T *z : {w.dx, w.dy, w.bx, w.by}) {
            k_fill<T><<<vbc, kVecThreads, 0, s>>>(z, T(0), cnt);
            SCT_TRY(check_launch("k_fill"));
        }
        // r = (data term) - A u
        SCT_TRY(data_rhs(w.cg.r));
        if (P.flags & RADON_SB_WARM) {
            SCT_TRY((apply_A_into_q<T>(op, A, u, batch, w.cg, s)));
            k_sub<T><<<vbc, kVecThreads, 0, s>>>(w.cg.r, w.cg.q, w.cg.r, cnt);
            SCT_TRY(check_launch("k_sub"));
        } else {
            k_fill<T><<<vbc, kVecThreads, 0, s>>>(u, T(0), cnt);
            SCT_TRY(check_launch("k_fill"));
        }
    }
    k_sb_reset<<<unsigned((batch + 63) / 64), 64, 0, s>>>(w.sbs, batch);
    SCT_TRY(check_launch("k_sb_reset"));
    const T thresh = T(1.0 / lambda);
    for (int k = 0; k < P.n_outer; ++k) {
        SCT_TRY((cg_run<T>(op, A, u, batch, P.n_cg, 0.0, w.cg, u, w.uprev, w.sbs, s)));
        k_sb_shrink<T><<<dim3(unsigned(vb), unsigned(batch)), kVecThreads, 0, s>>>(
            u, w.uprev, w.dx, w.dy, w.bx, w.by, w.dwx, w.dwy, thresh, w.sbs, w.part, op.n, op.nn);
        SCT_TRY(check_launch("k_sb_shrink"));
        k_sb_carry<T><<<dim3(unsigned(vb), unsigned(batch)), kVecThreads, 0, s>>>(
            w.cg.r, w.dwx, w.dwy, T(lambda), w.sbs, op.n, op.nn);
        SCT_TRY(check_launch("k_sb_carry"));
        k_sb_update<<<unsigned(batch), 256, 0, s>>>(w.part, vb, w.sbs,
                                                    final_state(w.cg.st, P.n_cg, batch), P.tol);
        SCT_TRY(check_launch("k_sb_update"));
    }
    if (info) {
        k_sb_info<<<unsigned((batch + 63) / 64), 64, 0, s>>>(w.sbs, info, batch);
        SCT_TRY(check_launch("k_sb_info"));
    }
    return RADON_OK;
}

template <class TM, class T>
static int sb_typed(const Op &op, const Sur *sur, const radon_sb_params &P, const void *f_v,
                    void *mu_v, int batch, void *ws, radon_sb_info *info, hipStream_t s)
{
    // data term alpha (MR)^T f through the stored adjoint
    auto rhs = [&](T *r) {
        return launch_adj<TM, T>(op, static_cast<const T *>(f_v), nullptr, r, P.alpha, 0.0, 0.0,
                                 nullptr, batch, s);
    };
    if (sur)
        return sb_run<T>(op, SurA<T>{*sur, P.alpha, P.lambda, 0.0}, rhs, P, mu_v, batch, ws, info, s);
    return sb_run<T>(op, ExactA<TM, T>{op, P.alpha, P.lambda, 0.0}, rhs, P, mu_v, batch, ws, info, s);
}


// ---------------------------------------------------------------------------
// Chambolle-Pock primal-dual TV (the method whose primal step is eq:PD_resolve)
// ---------------------------------------------------------------------------

// y <- clip(y + sigma K ubar, -1, 1) per component (anisotropic TV dual)
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_pd_dual(const T *__restrict__ ub,
                                                          T *__restrict__ yx, T *__restrict__ yy,
                                                          T sigma, int n, int64_t nn)
{
    const int64_t off = int64_t(blockIdx.y) * nn;
    for (int64_t i = int64_t(blockIdx.x) * kVecThreads + threadIdx.x; i < nn;
         i += int64_t(gridDim.x) * kVecThreads) {
        const int iy = int(i / n), ix = int(i % n);
        const int64_t j = off + i;
        const T u = ub[j];
        const T gx = ix < n - 1 ? ub[j + 1] - u : T(0);
        const T gy = iy < n - 1 ? ub[j + n] - u : T(0);
        yx[j] = fmin(fmax(yx[j] + sigma * gx, T(-1)), T(1));
        yy[j] = fmin(fmax(yy[j] + sigma * gy, T(-1)), T(1));
    }
}

// r <- u - tau K^T y + g (the right-hand side of eq:PD_resolve, g = tau alpha
// (MR)^T f); uo <- u
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_pd_rhs(const T *__restrict__ u,
                                                         const T *__restrict__ yx,
                                                         const T *__restrict__ yy,
                                                         const T *__restrict__ g, T tau,
                                                         T *__restrict__ r, T *__restrict__ uo,
                                                         int n, int64_t nn)
{
    const int64_t off = int64_t(blockIdx.y) * nn;
    for (int64_t i = int64_t(blockIdx.x) * kVecThreads + threadIdx.x; i < nn;
         i += int64_t(gridDim.x) * kVecThreads) {
        const int iy = int(i / n), ix = int(i % n);
        const int64_t j = off + i;
        T kt = T(0);
        if (ix >= 1) kt += yx[j - 1];
        if (ix <= n - 2) kt -= yx[j];
        if (iy >= 1) kt += yy[j - n];
        if (iy <= n - 2) kt -= yy[j];
        const T uj = u[j];
        r[j] = (uj - tau * kt) + g[j];
        uo[j] = uj;
    }
}

// ubar <- 2 u - uo (extrapolation with theta = 1)
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_pd_extrap(const T *__restrict__ u,
                                                            const T *__restrict__ uo,
                                                            T *__restrict__ ub, int64_t count)
{
    for (int64_t i = int64_t(blockIdx.x) * kVecThreads + threadIdx.x; i < count;
         i += int64_t(gridDim.x) * kVecThreads)
        ub[i] = T(2) * u[i] - uo[i];
}

template <class T>
struct PdBufs {
    CgBufs<T> cg;
    T *yx, *yy, *ub, *uo, *g;
};

template <class T>
static void carve_pd(const Op &op, int batch, Carver &c, PdBufs<T> &w)
{
    const int64_t nb = op.nn * batch;
    carve_cg(op, batch, c, w.cg);
    w.yx = c.take<T>(nb);
    w.yy = c.take<T>(nb);
    w.ub = c.take<T>(nb);
    w.uo = c.take<T>(nb);
    w.g = c.take<T>(nb);
}

int64_t pd_ws_bytes(const Op &op, int batch)
{
    Carver c(nullptr);
    if (op.vsize == 4) {
        PdBufs<float> w;
        carve_pd(op, batch, c, w);
    } else {
        PdBufs<double> w;
        carve_pd(op, batch, c, w);
    }
    return c.used;
}

template <class TM, class T>
static int pd_typed(const Op &op, const radon_pd_params &P, const void *f_v, void *mu_v, int batch,
                    void *ws, hipStream_t s)
{
    Carver c(ws);
    PdBufs<T> w;
    carve_pd(op, batch, c, w);
    const T *f = static_cast<const T *>(f_v);
    T *u = static_cast<T *>(mu_v);
    const int64_t cnt = op.nn * batch;
    const int vbc = vec_blocks(cnt), vb = vec_blocks(op.nn);
    const dim3 vg{unsigned(vb), unsigned(batch), 1u};
    const double ta = P.tau * P.alpha;
    const ExactA<TM, T> A{op, ta, 0.0, 1.0};   // I + tau alpha R^T M^T M R
    if (!(P.flags & RADON_SB_WARM)) {
        k_fill<T><<<vbc, kVecThreads, 0, s>>>(u, T(0), cnt);
        SCT_TRY(check_launch("k_fill"));
    }
    for (T *z : {w.yx, w.yy}) {
        k_fill<T><<<vbc, kVecThreads, 0, s>>>(z, T(0), cnt);
        SCT_TRY(check_launch("k_fill"));
    }
    k_copy<T><<<vbc, kVecThreads, 0, s>>>(u, w.ub, cnt);
    SCT_TRY(check_launch("k_copy"));
    SCT_TRY((launch_adj<TM, T>(op, f, nullptr, w.g, ta, 0.0, 0.0, nullptr, batch, s)));
    for (int k = 0; k < P.n_outer; ++k) {
        k_pd_dual<T><<<vg, kVecThreads, 0, s>>>(w.ub, w.yx, w.yy, T(P.sigma), op.n, op.nn);
        SCT_TRY(check_launch("k_pd_dual"));
        k_pd_rhs<T><<<vg, kVecThreads, 0, s>>>(u, w.yx, w.yy, w.g, T(P.tau), w.cg.r, w.uo, op.n,
                                                op.nn);
        SCT_TRY(check_launch("k_pd_rhs"));
        // CG from the current iterate with its true residual r = rhs - A u
        SCT_TRY((apply_A_into_q<T>(op, A, u, batch, w.cg, s)));
        k_sub<T><<<vbc, kVecThreads, 0, s>>>(w.cg.r, w.cg.q, w.cg.r, cnt);
        SCT_TRY(check_launch("k_sub"));
        SCT_TRY((cg_run<T>(op, A, u, batch, P.n_cg, 0.0, w.cg, nullptr, nullptr, nullptr, s)));
        k_pd_extrap<T><<<vbc, kVecThreads, 0, s>>>(u, w.uo, w.ub, cnt);
        SCT_TRY(check_launch("k_pd_extrap"));
    }
    return RADON_OK;
}

// ---------------------------------------------------------------------------
// Unrolled CG: forward with a checkpoint tape, and its vector-Jacobian product
// ---------------------------------------------------------------------------
// Forward: x_0 = 0, r_0 = rhs, n_iter CG iterations (an iteration with
// rho == 0 or a breakdown does nothing).  Every ckpt iterations the tape
// keeps (r, p, state).  The VJP maps dL/dx_n to dL/drhs by a reverse sweep
// through the iterations, one segment of ckpt iterations at a time: the
// segment is first replayed from its checkpoint (bitwise the same kernels,
// recording p_i, q_i = A p_i, r_{i+1} and the scalars), then reversed.
// Adjoints of one iteration (u_{i+1} = u_i + a p_i, r_{i+1} = r_i - a q_i,
// rho_{i+1} = <r_{i+1}, r_{i+1}>, beta = rho_{i+1}/rho_i, p_{i+1} = r_{i+1} +
// beta p_i, a = rho_i/gamma, gamma = <p_i, q_i>, q_i = A p_i with A symmetric):
//   betabar = <pbar, p_i>;  rbar += pbar;  pbar = beta pbar;
//   rhobar_{i+1} += betabar/rho_i;  rbar += 2 rhobar_{i+1} r_{i+1};
//   abar = <ubar, p_i> - <rbar, q_i>;  qbar = -a rbar;  pbar += a ubar;
//   rhobar_i = -betabar rho_{i+1}/rho_i^2 + abar/gamma;  gbar = -abar rho_i/gamma^2;
//   pbar += gbar q_i;  qbar += gbar p_i;  pbar += A qbar.
// and at the start p_0 = r_0 = rhs, rho_0 = <r_0, r_0>:
//   drhs = rbar + pbar + 2 rhobar_0 r_0.

struct IterRec {
    double rho, rho_next, a, gamma;
    int32_t active, pad[3];
};

struct RevScal {
    double carry;       // rhobar of the state after the step being reversed
    double betabar, up, rhobar_next;
};

__global__ void k_rec_scalars(const CgState *__restrict__ cur, const CgStep *__restrict__ stp,
                              const CgState *__restrict__ nxt, IterRec *__restrict__ rec, int batch)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    IterRec o;
    o.rho = cur[b].rho;
    o.rho_next = nxt[b].rho;
    o.a = stp[b].a;
    o.gamma = stp[b].gamma;
    o.active = stp[b].stopped ? 0 : 1;
    o.pad[0] = o.pad[1] = o.pad[2] = 0;
    rec[b] = o;
}

__global__ void k_state_copy(const CgState *__restrict__ src, CgState *__restrict__ dst, int batch)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < batch) dst[b] = src[b];
}

__global__ void k_rev_reset(RevScal *__restrict__ rs, int batch)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    RevScal z;
    z.carry = z.betabar = z.up = z.rhobar_next = 0.0;
    rs[b] = z;
}

// pbar += (A qbar of the later step); partials <pbar, p_i>, <ubar, p_i>.
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_rev_dots(T *__restrict__ pbar, T *__restrict__ aqb,
                                                           const T *__restrict__ p,
                                                           const T *__restrict__ ubar,
                                                           const IterRec *__restrict__ rec,
                                                           double *__restrict__ part, int64_t nn)
{
    __shared__ double red[kVecThreads];
    const int64_t b = blockIdx.y;
    const bool active = rec[b].active != 0;
    const int64_t off = b * nn;
    double d1 = 0.0, d2 = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kVecThreads + threadIdx.x; i < nn;
         i += int64_t(gridDim.x) * kVecThreads) {
        const int64_t j = off + i;
        const T pb = pbar[j] + aqb[j];
        pbar[j] = pb;
        if (!active) continue;
        d1 += double(pb) * double(p[j]);
        d2 += double(ubar[j]) * double(p[j]);
    }
    const double t1 = block_sum(d1, red);
    const double t2 = block_sum(d2, red);
    if (threadIdx.x == 0) {
        part[(b * gridDim.x + blockIdx.x) * 2 + 0] = t1;
        part[(b * gridDim.x + blockIdx.x) * 2 + 1] = t2;
    }
}

// rhobar_{i+1} = carry + betabar/rho_i; rbar += pbar + 2 rhobar_{i+1} r_{i+1};
// pbar *= beta; partial <rbar, q_i>.
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_rev_r(T *__restrict__ rbar, T *__restrict__ pbar,
                                                        const T *__restrict__ rn,
                                                        const T *__restrict__ q,
                                                        const IterRec *__restrict__ rec,
                                                        RevScal *__restrict__ rs,
                                                        const double *__restrict__ part_in,
                                                        int64_t n_in, double *__restrict__ part,
                                                        int64_t nn)
{
    __shared__ double red[kVecThreads];
    const int64_t b = blockIdx.y;
    const IterRec R = rec[b];
    if (!R.active) return;
    double v1 = 0.0, v2 = 0.0;
    for (int64_t i = threadIdx.x; i < n_in; i += kVecThreads) {
        v1 += part_in[(b * n_in + i) * 2 + 0];
        v2 += part_in[(b * n_in + i) * 2 + 1];
    }
    const double betabar = block_sum(v1, red);
    const double up = block_sum(v2, red);
    const double rhobar_next = rs[b].carry + betabar / R.rho;
    const double beta = R.rho_next / R.rho;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        RevScal o = rs[b];
        o.betabar = betabar;
        o.up = up;
        o.rhobar_next = rhobar_next;
        rs[b] = o;
    }
    const T two_rb = T(2.0 * rhobar_next), bt = T(beta);
    const int64_t off = b * nn;
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kVecThreads + threadIdx.x; i < nn;
         i += int64_t(gridDim.x) * kVecThreads) {
        const int64_t j = off + i;
        const T pb = pbar[j];
        const T rb = rbar[j] + pb + two_rb * rn[j];
        rbar[j] = rb;
        pbar[j] = bt * pb;
        acc += double(rb) * double(q[j]);
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) part[b * gridDim.x + blockIdx.x] = tot;
}

// abar = <ubar, p_i> - <rbar, q_i>; gbar = -abar rho_i/gamma^2;
// qbar = -a rbar + gbar p_i (and its transposed copy); pbar += a ubar + gbar q_i;
// the carried rhobar becomes rhobar_i.
template <class T>
__global__ __launch_bounds__(256) void k_rev_q(const T *__restrict__ rbar, T *__restrict__ pbar,
                                               T *__restrict__ qbar, T *__restrict__ qbarT,
                                               const T *__restrict__ p, const T *__restrict__ q,
                                               const T *__restrict__ ubar,
                                               const IterRec *__restrict__ rec,
                                               RevScal *__restrict__ rs,
                                               const double *__restrict__ part_in, int64_t n_in,
                                               int n, int64_t nn)
{
    __shared__ T tile[32][33];
    __shared__ double red[256];
    const int64_t b = blockIdx.z;
    const IterRec R = rec[b];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int64_t off = b * nn;
    if (!R.active) {
        // an inactive step passes every adjoint through: qbar = 0, so A qbar = 0
        for (int i = threadIdx.y; i < 32; i += 8) {
            const int iy = by + i, ix = bx + threadIdx.x;
            if (iy < n && ix < n) {
                qbar[off + int64_t(iy) * n + ix] = T(0);
                if (qbarT) qbarT[off + int64_t(ix) * n + iy] = T(0);
            }
        }
        return;
    }
    const int t = threadIdx.y * 32 + threadIdx.x;
    double v = 0.0;
    for (int64_t i = t; i < n_in; i += 256) v += part_in[b * n_in + i];
    const double rq = block_sum(v, red);
    const RevScal S = rs[b];
    const double abar = S.up - rq;
    const double gbar = -abar * R.rho / (R.gamma * R.gamma);
    if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0) {
        RevScal o = S;
        o.carry = -S.betabar * R.rho_next / (R.rho * R.rho) + abar / R.gamma;
        rs[b] = o;
    }
    const T a = T(R.a), g = T(gbar);
    for (int i = threadIdx.y; i < 32; i += 8) {
        const int iy = by + i, ix = bx + threadIdx.x;
        if (iy < n && ix < n) {
            const int64_t j = off + int64_t(iy) * n + ix;
            const T qb = -a * rbar[j] + g * p[j];
            qbar[j] = qb;
            pbar[j] = pbar[j] + a * ubar[j] + g * q[j];
            tile[i][threadIdx.x] = qb;
        }
    }
    if (!qbarT) return;
    __syncthreads();
    for (int i = threadIdx.y; i < 32; i += 8) {
        const int ix = bx + i, iy = by + threadIdx.x;
        if (ix < n && iy < n) qbarT[off + int64_t(ix) * n + iy] = tile[threadIdx.x][i];
    }
}

// drhs = rbar + pbar + (A qbar of step 0) + 2 rhobar_0 rhs
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_rev_final(const T *__restrict__ rbar,
                                                            const T *__restrict__ pbar,
                                                            const T *__restrict__ aqb,
                                                            const T *__restrict__ rhs,
                                                            const RevScal *__restrict__ rs,
                                                            T *__restrict__ out, int64_t nn)
{
    const int64_t b = blockIdx.y;
    const T two_r = T(2.0 * rs[b].carry);
    const int64_t off = b * nn;
    for (int64_t i = int64_t(blockIdx.x) * kVecThreads + threadIdx.x; i < nn;
         i += int64_t(gridDim.x) * kVecThreads) {
        const int64_t j = off + i;
        out[j] = rbar[j] + pbar[j] + aqb[j] + two_r * rhs[j];
    }
}

template <class T>
struct Tape {
    T *r = nullptr, *p = nullptr;   // [nseg][batch][nn]
    CgState *st = nullptr;          // [nseg][batch]
};

static int n_segments(int n_iter, int ckpt) { return n_iter <= 0 ? 0 : (n_iter + ckpt - 1) / ckpt; }

template <class T>
static void carve_tape(const Op &op, int batch, int n_iter, int ckpt, Carver &c, Tape<T> &t)
{
    const int64_t ns = n_segments(n_iter, ckpt);
    t.r = c.take<T>(ns * op.nn * batch);
    t.p = c.take<T>(ns * op.nn * batch);
    t.st = c.take<CgState>(ns * batch);
}

template <class T>
struct VjpBufs {
    CgBufs<T> cg;
    T *rec_p, *rec_q, *rec_r;            // [ckpt][batch][nn]
    IterRec *rec;                        // [ckpt][batch]
    T *pbar, *rbar, *qbar, *qbarT, *aqb;
    double *part;                        // [batch][vec_blocks][2]
    RevScal *rs;
};

template <class T>
static void carve_vjp(const Op &op, int batch, int ckpt, Carver &c, VjpBufs<T> &w)
{
    const int64_t nb = op.nn * batch;
    carve_cg(op, batch, c, w.cg);
    w.rec_p = c.take<T>(int64_t(ckpt) * nb);
    w.rec_q = c.take<T>(int64_t(ckpt) * nb);
    w.rec_r = c.take<T>(int64_t(ckpt) * nb);
    w.rec = c.take<IterRec>(int64_t(ckpt) * batch);
    w.pbar = c.take<T>(nb);
    w.rbar = c.take<T>(nb);
    w.qbar = c.take<T>(nb);
    w.qbarT = op.need_T ? c.take<T>(nb) : nullptr;
    w.aqb = c.take<T>(nb);
    w.part = c.take<double>(int64_t(2) * vec_blocks(op.nn) * batch);
    w.rs = c.take<RevScal>(batch);
}

static int64_t unrolled_bytes(const Op &op, int which, int n_iter, int ckpt, int batch)
{
    Carver c(nullptr);
    if (op.vsize == 4) {
        if (which == 0) { Tape<float> t; carve_tape(op, batch, n_iter, ckpt, c, t); }
        else { VjpBufs<float> w; carve_vjp(op, batch, ckpt, c, w); }
    } else {
        if (which == 0) { Tape<double> t; carve_tape(op, batch, n_iter, ckpt, c, t); }
        else { VjpBufs<double> w; carve_vjp(op, batch, ckpt, c, w); }
    }
    return c.used;
}

template <class TM, class T>
static int unrolled_fwd_typed(const Op &op, double alpha, double lambda, double sigma,
                              const T *rhs, T *x, int batch, int n_iter, int ckpt, void *tape_mem,
                              void *ws, hipStream_t s)
{
    Carver tc(tape_mem);
    Tape<T> tape;
    carve_tape(op, batch, n_iter, ckpt, tc, tape);
    Carver c(ws);
    CgBufs<T> w;
    carve_cg(op, batch, c, w);
    const int64_t cnt = op.nn * batch;
    const int vbc = vec_blocks(cnt);
    k_fill<T><<<vbc, kVecThreads, 0, s>>>(x, T(0), cnt);
    k_copy<T><<<vbc, kVecThreads, 0, s>>>(rhs, w.r, cnt);
    SCT_TRY(check_launch("k_copy"));
    SCT_TRY(cg_start<T>(op, batch, w, nullptr, nullptr, nullptr, s));
    for (int it = 0; it < n_iter; ++it) {
        if (it % ckpt == 0) {
            const int64_t sg = it / ckpt;
            k_copy<T><<<vbc, kVecThreads, 0, s>>>(w.r, tape.r + sg * cnt, cnt);
            k_copy<T><<<vbc, kVecThreads, 0, s>>>(w.p, tape.p + sg * cnt, cnt);
            k_state_copy<<<unsigned((batch + 63) / 64), 64, 0, s>>>(w.st + int64_t(it & 1) * batch,
                                                                   tape.st + sg * batch, batch);
            SCT_TRY(check_launch("tape"));
        }
        SCT_TRY((cg_iter<T>(op, ExactA<TM, T>{op, alpha, lambda, sigma}, x, batch, it, 0.0, w, s)));
    }
    return RADON_OK;
}

template <class TM, class T>
static int unrolled_vjp_typed(const Op &op, double alpha, double lambda, double sigma,
                              const void *tape_mem, const T *gx, T *grhs, int batch, int n_iter,
                              int ckpt, void *ws, hipStream_t s)
{
    Carver tc(const_cast<void *>(tape_mem));
    Tape<T> tape;
    carve_tape(op, batch, n_iter, ckpt, tc, tape);
    Carver c(ws);
    VjpBufs<T> w;
    carve_vjp(op, batch, ckpt, c, w);
    const int64_t cnt = op.nn * batch;
    const int vbc = vec_blocks(cnt), vb = vec_blocks(op.nn);
    const unsigned t = unsigned(tiles_of(op.n));
    const dim3 tg{t, t, unsigned(batch)}, tb{32, 8, 1};
    const unsigned sb = unsigned((batch + 63) / 64);
    for (T *z : {w.pbar, w.rbar, w.aqb}) k_fill<T><<<vbc, kVecThreads, 0, s>>>(z, T(0), cnt);
    k_rev_reset<<<sb, 64, 0, s>>>(w.rs, batch);
    SCT_TRY(check_launch("k_rev_reset"));
    for (int sg = n_segments(n_iter, ckpt) - 1; sg >= 0; --sg) {
        const int k0 = sg * ckpt, k1 = (k0 + ckpt < n_iter) ? k0 + ckpt : n_iter;
        // replay the segment from its checkpoint, recording what the reverse needs
        k_copy<T><<<vbc, kVecThreads, 0, s>>>(tape.r + int64_t(sg) * cnt, w.cg.r, cnt);
        k_copy<T><<<vbc, kVecThreads, 0, s>>>(tape.p + int64_t(sg) * cnt, w.cg.p, cnt);
        if (w.cg.pT) SCT_TRY(launch_transpose<T>(op, w.cg.p, w.cg.pT, batch, s));
        k_state_copy<<<sb, 64, 0, s>>>(tape.st + int64_t(sg) * batch, w.cg.st + int64_t(k0 & 1) * batch,
                                       batch);
        SCT_TRY(check_launch("replay"));
        for (int it = k0; it < k1; ++it) {
            const int64_t o = int64_t(it - k0) * cnt;
            SCT_TRY((cg_iter<T>(op, ExactA<TM, T>{op, alpha, lambda, sigma}, nullptr, batch, it, 0.0,
                                w.cg, s, w.rec_q + o, w.rec_p + o, w.rec_r + o)));
            k_rec_scalars<<<sb, 64, 0, s>>>(w.cg.st + int64_t(it & 1) * batch,
                                            w.cg.step + int64_t(it & 1) * batch,
                                            w.cg.st + int64_t((it + 1) & 1) * batch,
                                            w.rec + int64_t(it - k0) * batch, batch);
            SCT_TRY(check_launch("k_rec_scalars"));
        }
        // reverse through the segment
        for (int it = k1 - 1; it >= k0; --it) {
            const int64_t o = int64_t(it - k0) * cnt;
            const IterRec *R = w.rec + int64_t(it - k0) * batch;
            const T *p_i = w.rec_p + o, *q_i = w.rec_q + o, *r_n = w.rec_r + o;
            k_rev_dots<T><<<dim3(unsigned(vb), unsigned(batch)), kVecThreads, 0, s>>>(
                w.pbar, w.aqb, p_i, gx, R, w.part, op.nn);
            SCT_TRY(check_launch("k_rev_dots"));
            k_rev_r<T><<<dim3(unsigned(vb), unsigned(batch)), kVecThreads, 0, s>>>(
                w.rbar, w.pbar, r_n, q_i, R, w.rs, w.part, vb, w.cg.part_vec, op.nn);
            SCT_TRY(check_launch("k_rev_r"));
            k_rev_q<T><<<tg, tb, 0, s>>>(w.rbar, w.pbar, w.qbar, w.qbarT, p_i, q_i, gx, R, w.rs,
                                         w.cg.part_vec, vb, op.n, op.nn);
            SCT_TRY(check_launch("k_rev_q"));
            // A qbar, added to pbar by the next (earlier) step or the final kernel;
            // the products' scratch follows y (see carve_cg)
            T *scr = w.cg.y + op.rows * batch;
            SCT_TRY((launch_fwd<TM, T>(op, w.qbar, w.qbarT, w.cg.y, batch, s,
                                       fwd_part_elems(op, batch) ? scr : nullptr)));
            SCT_TRY((launch_adj<TM, T>(op, w.cg.y, w.qbar, w.aqb, alpha, lambda, sigma, nullptr,
                                       batch, s, adj_scratch_elems(op, batch) ? scr : nullptr)));
        }
    }
    // r_0 = rhs is the first checkpoint's residual (x_0 = 0)
    k_rev_final<T><<<dim3(unsigned(vb), unsigned(batch)), kVecThreads, 0, s>>>(
        w.rbar, w.pbar, w.aqb, tape.r, w.rs, grhs, op.nn);
    return check_launch("k_rev_final");
}

}  // namespace sct

using namespace sct;

extern "C" int cg_solve(const radon_op *p, double alpha, double lambda, double sigma,
                        const void *rhs, void *x, int32_t x0_given, int32_t batch, int32_t layout,
                        int32_t n_iter, double rtol, void *ws, int64_t ws_bytes, radon_cg_info *info,
                        void *stream)
{
    clear_error();
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    SCT_TRY(check_layout(layout));
    if (!rhs || !x) return set_error(RADON_EINVAL, "rhs and x must be non-NULL");
    if (rhs == x) return set_error(RADON_EINVAL, "x must not alias rhs");
    if (n_iter < 0) return set_error(RADON_EINVAL, "n_iter must be >= 0 (got %d)", n_iter);
    if (!(rtol >= 0.0)) return set_error(RADON_EINVAL, "rtol must be >= 0");
    const Op &op = *as_op(p);
    const int64_t base = cg_ws_bytes(op, batch);
    const bool relay = relays(layout, batch);
    SCT_TRY(check_ws(ws, ws_bytes, base + (relay ? pixel_layout_extra(op, RADON_WS_CG, batch) : 0), "cg_solve"));
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        if (!relay)
            return cg_typed<TM, TV>(op, alpha, lambda, sigma, rhs, x, x0_given, batch, n_iter, rtol, ws,
                                    info, s);
        TV *ri = nullptr, *xi = nullptr;
        relay_buffers<TV>(ws, base, op.nn * batch, op.nn * batch, &ri, &xi);
        SCT_TRY(launch_relayout<TV>(static_cast<const TV *>(rhs), ri, op.nn, batch, false, s));
        if (x0_given) SCT_TRY(launch_relayout<TV>(static_cast<const TV *>(x), xi, op.nn, batch, false, s));
        SCT_TRY((cg_typed<TM, TV>(op, alpha, lambda, sigma, ri, xi, x0_given, batch, n_iter, rtol, ws,
                                  info, s)));
        return launch_relayout<TV>(xi, static_cast<TV *>(x), op.nn, batch, true, s);
    });
}

extern "C" int split_bregman_tv(const radon_op *p, const radon_sb_params *params, const void *f,
                                void *mu, int32_t batch, int32_t layout, void *ws, int64_t ws_bytes,
                                radon_sb_info *info, void *stream)
{
    clear_error();
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    SCT_TRY(check_layout(layout));
    if (!params) return set_error(RADON_EINVAL, "params is NULL");
    if (!f || !mu) return set_error(RADON_EINVAL, "f and mu must be non-NULL");
    if (!(params->lambda > 0.0)) return set_error(RADON_EINVAL, "lambda must be > 0");
    if (params->n_outer < 0 || params->n_cg < 0)
        return set_error(RADON_EINVAL, "n_outer and n_cg must be >= 0");
    if (!(params->tol >= 0.0)) return set_error(RADON_EINVAL, "tol must be >= 0");
    if (params->flags & ~(RADON_SB_WARM | RADON_SB_RESUME))
        return set_error(RADON_EINVAL, "unknown flags 0x%x", params->flags);
    const Op &op = *as_op(p);
    const int64_t base = sb_ws_bytes(op, batch);
    const bool relay = relays(layout, batch);
    SCT_TRY(check_ws(ws, ws_bytes, base + (relay ? pixel_layout_extra(op, RADON_WS_SB, batch) : 0),
                     "split_bregman_tv"));
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        if (!relay) return sb_typed<TM, TV>(op, nullptr, *params, f, mu, batch, ws, info, s);
        TV *ui = nullptr, *fi = nullptr;
        relay_buffers<TV>(ws, base, op.nn * batch, op.rows * batch, &ui, &fi);
        SCT_TRY(launch_relayout<TV>(static_cast<const TV *>(f), fi, op.rows, batch, false, s));
        if (params->flags & (RADON_SB_WARM | RADON_SB_RESUME))
            SCT_TRY(launch_relayout<TV>(static_cast<const TV *>(mu), ui, op.nn, batch, false, s));
        SCT_TRY((sb_typed<TM, TV>(op, nullptr, *params, fi, ui, batch, ws, info, s)));
        return launch_relayout<TV>(ui, static_cast<TV *>(mu), op.nn, batch, true, s);
    });
}

extern "C" int split_bregman_tv_surrogate(const radon_op *p, const radon_surrogate *sp,
                                          const radon_sb_params *params, const void *f, void *mu,
                                          int32_t batch, void *ws, int64_t ws_bytes,
                                          radon_sb_info *info, void *stream)
{
    clear_error();
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    if (!params) return set_error(RADON_EINVAL, "params is NULL");
    if (!f || !mu) return set_error(RADON_EINVAL, "f and mu must be non-NULL");
    if (!(params->lambda > 0.0)) return set_error(RADON_EINVAL, "lambda must be > 0");
    if (params->n_outer < 0 || params->n_cg < 0)
        return set_error(RADON_EINVAL, "n_outer and n_cg must be >= 0");
    if (!(params->tol >= 0.0)) return set_error(RADON_EINVAL, "tol must be >= 0");
    if (params->flags & ~(RADON_SB_WARM | RADON_SB_RESUME))
        return set_error(RADON_EINVAL, "unknown flags 0x%x", params->flags);
    const Op &op = *as_op(p);
    if (!sp) return set_error(RADON_EINVAL, "surrogate is NULL");
    const Sur &sur = *reinterpret_cast<const Sur *>(sp);
    if (sur.n != op.n || sur.dtype != op.dtype)
        return set_error(RADON_EINVAL, "the surrogate belongs to an operator of another size or dtype");
    SCT_TRY(check_ws(ws, ws_bytes, sb_ws_bytes(op, batch), "split_bregman_tv_surrogate"));
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        return sb_typed<TM, TV>(op, &sur, *params, f, mu, batch, ws, info, s);
    });
}

namespace sct {
int capture_graph(const std::function<int(hipStream_t)> &body, radon_graph **out);
}

extern "C" int split_bregman_tv_graph(const radon_op *p, const radon_sb_params *params,
                                      const void *f, void *mu, int32_t batch, void *ws,
                                      int64_t ws_bytes, radon_sb_info *info, radon_graph **out)
{
    clear_error();
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    *out = nullptr;
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    if (!params) return set_error(RADON_EINVAL, "params is NULL");
    if (!f || !mu) return set_error(RADON_EINVAL, "f and mu must be non-NULL");
    if (!(params->lambda > 0.0)) return set_error(RADON_EINVAL, "lambda must be > 0");
    if (params->n_outer < 0 || params->n_cg < 0)
        return set_error(RADON_EINVAL, "n_outer and n_cg must be >= 0");
    if (!(params->tol >= 0.0)) return set_error(RADON_EINVAL, "tol must be >= 0");
    if (params->flags & ~RADON_SB_WARM)
        return set_error(RADON_EINVAL, "flags 0x%x: only RADON_SB_WARM can be captured", params->flags);
    const Op &op = *as_op(p);
    SCT_TRY(check_ws(ws, ws_bytes, sb_ws_bytes(op, batch), "split_bregman_tv_graph"));
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    const radon_sb_params P = *params;
    return capture_graph(
        [&](hipStream_t cs) {
            return dispatch(op, [&](auto *tm, auto *tv) {
                SCT_TYPES(tm, tv);
                return sb_typed<TM, TV>(op, nullptr, P, f, mu, batch, ws, info, cs);
            });
        },
        out);
}

extern "C" int split_bregman_tv_fourier(const radon_fourier *fp, int32_t path,
                                        const radon_sb_params *params, const void *fhat, void *mu,
                                        int32_t batch, void *ws, int64_t ws_bytes,
                                        radon_sb_info *info, void *stream)
{
    clear_error();
    if (!fp) return set_error(RADON_EINVAL, "Fourier operator is NULL");
    SCT_TRY(check_batch(batch));
    if (!params) return set_error(RADON_EINVAL, "params is NULL");
    if (!fhat || !mu) return set_error(RADON_EINVAL, "fhat and mu must be non-NULL");
    if (path != RADON_FOURIER_FUSED && path != RADON_FOURIER_NUFFT)
        return set_error(RADON_EINVAL, "unknown path %d", path);
    if (!(params->lambda > 0.0)) return set_error(RADON_EINVAL, "lambda must be > 0");
    if (params->n_outer < 0 || params->n_cg < 0)
        return set_error(RADON_EINVAL, "n_outer and n_cg must be >= 0");
    if (!(params->tol >= 0.0)) return set_error(RADON_EINVAL, "tol must be >= 0");
    if (params->flags & ~(RADON_SB_WARM | RADON_SB_RESUME))
        return set_error(RADON_EINVAL, "unknown flags 0x%x", params->flags);
    const Fou &fou = *reinterpret_cast<const Fou *>(fp);
    const Op &op = *fou.op;
    if (fourier_parts(fou) > std::max<int64_t>(op.n_ag, op.n))
        return set_error(RADON_EUNSUPPORTED, "more Fourier partials than the solver buffers hold");
    Carver c(ws);
    c.take<char>(sb_ws_bytes(op, batch));
    void *grids = c.take<char>(fourier_grid_bytes(fou, batch));
    SCT_TRY(check_ws(ws, ws_bytes, c.used, "split_bregman_tv_fourier"));
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const radon_sb_params &P = *params;
    return dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        auto rhs = [&](TV *r) {
            return launch_fourier_adj<TM, TV>(fou, static_cast<const TV *>(fhat), r, P.alpha, batch,
                                              grids, s);
        };
        return sb_run<TV>(op, FouA<TM, TV>{fou, path, P.alpha, P.lambda, 0.0, grids}, rhs, P, mu,
                          batch, ws, info, s);
    });
}

extern "C" int radon_unrolled_sizes(const radon_op *p, int32_t n_iter, int32_t ckpt, int32_t batch,
                                    int64_t *tape_bytes, int64_t *ws_fwd_bytes,
                                    int64_t *ws_vjp_bytes)
{
    clear_error();
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    if (n_iter < 0) return set_error(RADON_EINVAL, "n_iter must be >= 0 (got %d)", n_iter);
    if (ckpt < 1) return set_error(RADON_EINVAL, "ckpt must be >= 1 (got %d)", ckpt);
    const Op &op = *as_op(p);
    const int k = ckpt < n_iter ? ckpt : (n_iter > 0 ? n_iter : 1);
    if (tape_bytes) *tape_bytes = unrolled_bytes(op, 0, n_iter, ckpt, batch);
    if (ws_fwd_bytes) *ws_fwd_bytes = cg_ws_bytes(op, batch);
    if (ws_vjp_bytes) *ws_vjp_bytes = unrolled_bytes(op, 1, n_iter, k, batch);
    return RADON_OK;
}

static int check_unrolled(const radon_op *p, int32_t batch, int32_t n_iter, int32_t ckpt,
                          const void *tape, int64_t tape_bytes)
{
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    if (n_iter < 0) return set_error(RADON_EINVAL, "n_iter must be >= 0 (got %d)", n_iter);
    if (ckpt < 1) return set_error(RADON_EINVAL, "ckpt must be >= 1 (got %d)", ckpt);
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    const int64_t need = unrolled_bytes(*as_op(p), 0, n_iter, ckpt, batch);
    if (need > 0 && !tape) return set_error(RADON_EWORKSPACE, "tape is NULL (%lld bytes needed)",
                                            (long long)need);
    if (tape_bytes < need)
        return set_error(RADON_EWORKSPACE, "tape of %lld bytes, %lld needed", (long long)tape_bytes,
                         (long long)need);
    return RADON_OK;
}

extern "C" int cg_unrolled(const radon_op *p, double alpha, double lambda, double sigma,
                           const void *rhs, void *x, int32_t batch, int32_t n_iter, int32_t ckpt,
                           void *tape, int64_t tape_bytes, void *ws, int64_t ws_bytes,
                           void *stream)
{
    clear_error();
    SCT_TRY(check_unrolled(p, batch, n_iter, ckpt, tape, tape_bytes));
    if (!rhs || !x) return set_error(RADON_EINVAL, "rhs and x must be non-NULL");
    if (rhs == x) return set_error(RADON_EINVAL, "x must not alias rhs");
    const Op &op = *as_op(p);
    SCT_TRY(check_ws(ws, ws_bytes, cg_ws_bytes(op, batch), "cg_unrolled"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    return dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        return unrolled_fwd_typed<TM, TV>(op, alpha, lambda, sigma, static_cast<const TV *>(rhs),
                                          static_cast<TV *>(x), batch, n_iter, ckpt, tape, ws, s);
    });
}

extern "C" int cg_unrolled_vjp(const radon_op *p, double alpha, double lambda, double sigma,
                               const void *tape, int64_t tape_bytes, const void *gx, void *grhs,
                               int32_t batch, int32_t n_iter, int32_t ckpt, void *ws,
                               int64_t ws_bytes, void *stream)
{
    clear_error();
    SCT_TRY(check_unrolled(p, batch, n_iter, ckpt, tape, tape_bytes));
    if (!gx || !grhs) return set_error(RADON_EINVAL, "gx and grhs must be non-NULL");
    const Op &op = *as_op(p);
    const int k = ckpt < n_iter ? ckpt : (n_iter > 0 ? n_iter : 1);
    SCT_TRY(check_ws(ws, ws_bytes, unrolled_bytes(op, 1, n_iter, k, batch), "cg_unrolled_vjp"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n_iter == 0) {
        // x = 0 whatever the rhs: the gradient is zero
        const int64_t cnt = op.nn * batch;
        if (op.vsize == 4)
            k_fill<float><<<vec_blocks(cnt), kVecThreads, 0, s>>>(static_cast<float *>(grhs), 0.f, cnt);
        else
            k_fill<double><<<vec_blocks(cnt), kVecThreads, 0, s>>>(static_cast<double *>(grhs), 0.0, cnt);
        return check_launch("k_fill");
    }
    return dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        return unrolled_vjp_typed<TM, TV>(op, alpha, lambda, sigma, tape,
                                          static_cast<const TV *>(gx), static_cast<TV *>(grhs),
                                          batch, n_iter, k, ws, s);
    });
}

extern "C" int chambolle_pock_tv(const radon_op *p, const radon_pd_params *params, const void *f,
                                 void *mu, int32_t batch, void *ws, int64_t ws_bytes, void *stream)
{
    clear_error();
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    if (!params) return set_error(RADON_EINVAL, "params is NULL");
    if (!f || !mu) return set_error(RADON_EINVAL, "f and mu must be non-NULL");
    if (!(params->tau > 0.0) || !(params->sigma > 0.0))
        return set_error(RADON_EINVAL, "tau and sigma must be > 0");
    if (!(params->alpha >= 0.0)) return set_error(RADON_EINVAL, "alpha must be >= 0");
    if (params->n_outer < 0 || params->n_cg < 0)
        return set_error(RADON_EINVAL, "n_outer and n_cg must be >= 0");
    if (params->flags & ~RADON_SB_WARM) return set_error(RADON_EINVAL, "unknown flags 0x%x", params->flags);
    const Op &op = *as_op(p);
    SCT_TRY(check_ws(ws, ws_bytes, pd_ws_bytes(op, batch), "chambolle_pock_tv"));
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        return pd_typed<TM, TV>(op, *params, f, mu, batch, ws, s);
    });
}
