// Several operators of different geometry (an uneven mixed batch: image
// sizes, angle counts and bin counts differ per instance) applied and solved
// together.  Every phase of a product or of a CG iteration is ONE launch over
// all instances: the work items of the instances (ray bundles, 8x8 adjoint
// tiles, 32x32 vector tiles, vector blocks) are concatenated into one index
// space and each workgroup finds its instance by a binary search over the
// instances' first items.  Vectors of all instances are packed back to back.
// The per-instance operator is A_i = alpha_i R_i^T M_i^T M_i R_i +
// lambda_i K^T K + sigma_i I (Section 2), with the weights fixed when the
// group is created.  A whole CG solve can be captured once into a HIP graph
// and replayed with one launch.
#include "cg.hpp"
#include "products.hpp"

#include <functional>

#include <algorithm>
#include <new>

namespace sct {

// Device descriptor of one instance.
struct MultiInst {
    const FwdBundle *fb;
    const uint16_t *f_idx;
    const void *f_v0, *f_v1;
    const RayEdge *f_edge;
    const uint8_t *a_rel;
    const uint16_t *a_base;
    const void *a_v0, *a_v1;
    int64_t n_ag, nn, rows;
    int64_t img_off, sino_off;   // element offsets in the packed image / sinogram vectors
    int64_t part_off;            // element offset of the band partials (banded forward)
    double alpha, lambda, sigma;
    int32_t n, n_meas, n_aq, nb, tiles8, tiles32, need_T;
    int32_t n_bands;             // > 0: the forward entries are (bundle, band) items
};

struct Multi {
    int count = 0, dtype = 0, vsize = 0;
    int bw = kFwdLanes;                       // bundle width shared by every instance
    std::vector<const Op *> ops;
    std::vector<int64_t> img_off, sino_off;   // host, count + 1 entries
    std::vector<int64_t> part_off;            // host: band partial offset, -1 if not banded
    MultiInst *inst = nullptr;                // device [count]
    int2 *fwork = nullptr;                    // device (instance, bundle); bundle -1 = padding;
                                              // (instance, band << 24 | bundle) for banded instances
    int64_t n_fwork = 0;
    int64_t n_fpart = 0;                      // band partial elements of all banded instances
    int64_t *grp_start = nullptr;             // device [count + 1]: first adjoint tile group
    int64_t *t32_start = nullptr;             // device [count + 1]: first 32x32 vector tile
    int64_t *vb_start = nullptr;              // device [count + 1]: first vector block
    int64_t n_grp = 0, n_t32 = 0, n_vb = 0;
    bool any_T = false;
    int adj_w = 2;
    std::vector<void *> owned;
};

struct Graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// index of the instance whose item range [start[i], start[i+1]) holds g
__device__ inline int find_inst(const int64_t *__restrict__ start, int count, int64_t g)
{
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// product kernels
// ---------------------------------------------------------------------------

// xT = transposed copy of the instances whose measured angles need it
template <class T>
__global__ __launch_bounds__(256) void k_multi_transpose(const T *__restrict__ x, T *__restrict__ xT,
                                                         const MultiInst *__restrict__ inst,
                                                         const int64_t *__restrict__ t32_start,
                                                         int count)
{
    __shared__ T tile[32][33];
    const int i = find_inst(t32_start, count, blockIdx.x);
    const MultiInst &I = inst[i];
    if (!I.need_T) return;
    const int64_t t = int64_t(blockIdx.x) - t32_start[i];
    const int bx = int(t % I.tiles32) * 32, by = int(t / I.tiles32) * 32, n = I.n;
    const T *__restrict__ xi = x + I.img_off;
    T *__restrict__ xo = xT + I.img_off;
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int iy = by + r, ix = bx + threadIdx.x;
        if (iy < n && ix < n) tile[r][threadIdx.x] = xi[int64_t(iy) * n + ix];
    }
    __syncthreads();
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int ix = bx + r, iy = by + threadIdx.x;
        if (ix < n && iy < n) xo[int64_t(ix) * n + iy] = tile[threadIdx.x][r];
    }
}

// Forward products of every instance over the concatenated (instance, bundle)
// list.  Each instance's segment keeps its XCD-aware order and starts at a
// multiple of 8; the grid is a multiple of 8, so block i runs on XCD i % 8 and
// takes only entries o with o % 8 == i % 8, as in the single-operator product.
// The entries are handed out in list order through one ticket counter per
// XCD: a static round-robin would let blocks drift apart over the instances,
// keeping many instances' images live in the caches at once.
template <class TM, class TV, int W, int BW>
__global__ __launch_bounds__(64 * W) void k_multi_fwd(const int2 *__restrict__ work, int64_t n_work,
                                                      const MultiInst *__restrict__ inst,
                                                      const TV *__restrict__ x,
                                                      const TV *__restrict__ xT, TV *__restrict__ y,
                                                      TV *__restrict__ part,
                                                      uint32_t *__restrict__ tickets)
{
    __shared__ int64_t next;
    const int xcd = int(blockIdx.x & 7u);
    uint32_t *const counter = tickets + xcd * kTicketStride;
    if (threadIdx.x == 0) next = 8 * int64_t(atomicAdd(counter, 1u)) + xcd;
    __syncthreads();
    int64_t o = next;
    while (o < n_work) {
        // the following ticket is taken now and read only after this bundle,
        // so the atomic's round trip overlaps the bundle's work
        uint32_t ticket = 0;
        if (threadIdx.x == 0) ticket = atomicAdd(counter, 1u);
        const int2 w = work[o];
        if (w.y >= 0) {   // uniform per block; padding entries carry no bundle
            const MultiInst &I = inst[w.x];
            if (I.n_bands > 0) {   // a (bundle, band) item, as in k_fwd_band
                const int band = w.y >> 24;
                const FwdBundle d = I.fb[w.y & 0xffffff];
                const int nq = d.nrows >> 2;
                const int lo = band * kBandLines - d.m0, hi = lo + kBandLines;
                const int tq0 = lo <= 0 ? 0 : min(nq, (lo + 3) >> 2);
                const int tq1 = hi <= 0 ? 0 : min(nq, (hi + 3) >> 2);
                fwd_bundle<TM, TV, W, 1, BW>(d, I.f_idx, static_cast<const TM *>(I.f_v0),
                                             static_cast<const TM *>(I.f_v1), I.f_edge,
                                             (d.horiz ? xT : x) + I.img_off,
                                             part + I.part_off + int64_t(band) * I.rows, I.n, I.nn,
                                             I.rows, 1, tq0, tq1);
            } else {
                const FwdBundle d = I.fb[w.y];
                fwd_bundle<TM, TV, W, 1, BW>(d, I.f_idx, static_cast<const TM *>(I.f_v0),
                                             static_cast<const TM *>(I.f_v1), I.f_edge,
                                             (d.horiz ? xT : x) + I.img_off, y + I.sino_off, I.n,
                                             I.nn, I.rows, 1);
            }
        }
        __syncthreads();   // every wave has read `next`
        if (threadIdx.x == 0) next = 8 * int64_t(ticket) + xcd;
        __syncthreads();
        o = next;
    }
}

// Adjoint products of every instance over the concatenated tile groups.
// normal = 0: out = (MR)^T y; normal = 1: out = A_i x with the instance's
// weights.  With part != nullptr each block leaves its share of <x, out> per
// instance in part[instance][gridDim.x] (0 for instances it has no tile of):
// a block meets the instances in increasing order, so it flushes its running
// sum whenever the instance changes.
template <class TM, class T, int W>
__global__ __launch_bounds__(64 * W) void k_multi_adj(const int64_t *__restrict__ grp_start,
                                                      int count, const MultiInst *__restrict__ inst,
                                                      const T *__restrict__ y,
                                                      const T *__restrict__ x, T *__restrict__ out,
                                                      int normal, double *__restrict__ part)
{
    using Q = typename Quad<TM>::type;
    __shared__ T band[W * 4 * kAdjBand];
    __shared__ uint16_t bases[W * kAdjLanes];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t n_grp = grp_start[count];
    const int64_t G = gridDim.x;
    int cur = -1;
    int64_t cur_lo = 0, cur_hi = 0;   // tile groups of instance cur
    double dsum = 0.0;
    for (int64_t g = blockIdx.x; g < n_grp; g += G) {
        if (g >= cur_hi) {   // g only grows: search when it leaves the current instance
            const int i = find_inst(grp_start, count, g);
            if (part && wave == 0) {
                if (cur >= 0) {
                    const double v = wave_sum(dsum);
                    if (lane == 0) part[int64_t(cur) * G + blockIdx.x] = v;
                }
                for (int k = cur + 1; k < i; ++k)
                    if (lane == 0) part[int64_t(k) * G + blockIdx.x] = 0.0;
            }
            cur = i;
            cur_lo = grp_start[i];
            cur_hi = grp_start[i + 1];
            dsum = 0.0;
        }
        const MultiInst &I = inst[cur];
        const int64_t gl = g - cur_lo;
        const T acc = adj_tile1<TM, T, W>(gl, reinterpret_cast<const uint32_t *>(I.a_rel), I.a_base,
                                          static_cast<const Q *>(I.a_v0),
                                          static_cast<const Q *>(I.a_v1), I.n_meas, I.n_aq, I.nb,
                                          y + I.sino_off, band, bases);
        if (wave == 0) {
            if (normal)
                dsum += adj_epilogue(gl, lane, acc, x + I.img_off, out + I.img_off, T(I.alpha),
                                     T(I.lambda), T(I.sigma), I.n, I.tiles8);
            else
                adj_epilogue(gl, lane, acc, static_cast<const T *>(nullptr), out + I.img_off, T(1),
                             T(0), T(0), I.n, I.tiles8);
        }
    }
    if (part && wave == 0) {
        if (cur >= 0) {
            const double v = wave_sum(dsum);
            if (lane == 0) part[int64_t(cur) * G + blockIdx.x] = v;
        }
        for (int k = cur + 1; k < count; ++k)
            if (lane == 0) part[int64_t(k) * G + blockIdx.x] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// CG kernels (same recurrences as the single-operator CG, one state per
// instance; every reduction in a fixed order)
// ---------------------------------------------------------------------------

// p = r (+ transposed copy), partial <r, r> per 32x32 tile
template <class T>
__global__ __launch_bounds__(256) void k_multi_cg_start(const T *__restrict__ r, T *__restrict__ p,
                                                        T *__restrict__ pT,
                                                        const MultiInst *__restrict__ inst,
                                                        const int64_t *__restrict__ t32_start,
                                                        int count, double *__restrict__ part)
{
    __shared__ T tile[32][33];
    __shared__ double red[256];
    const int i = find_inst(t32_start, count, blockIdx.x);
    const MultiInst &I = inst[i];
    const int64_t t = int64_t(blockIdx.x) - t32_start[i];
    const int bx = int(t % I.tiles32) * 32, by = int(t / I.tiles32) * 32, n = I.n;
    const int64_t off = I.img_off;
    double acc = 0.0;
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int iy = by + k, ix = bx + threadIdx.x;
        if (iy < n && ix < n) {
            const int64_t j = off + int64_t(iy) * n + ix;
            const T v = r[j];
            p[j] = v;
            tile[k][threadIdx.x] = v;
            acc += double(v) * double(v);
        }
    }
    const double tot = block_sum(acc, red);
    if (pT && I.need_T) {
        for (int k = threadIdx.y; k < 32; k += 8) {
            const int ix = bx + k, iy = by + threadIdx.x;
            if (ix < n && iy < n) pT[off + int64_t(ix) * n + iy] = tile[threadIdx.x][k];
        }
    }
    if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = tot;
}

// rho_0 of instance blockIdx.x; resets its state (ring slot 0)
__global__ __launch_bounds__(256) void k_multi_begin(const double *__restrict__ part,
                                                     const int64_t *__restrict__ t32_start,
                                                     CgState *__restrict__ st)
{
    __shared__ double red[256];
    const int i = blockIdx.x;
    const double rho = sum_part_block(part + t32_start[i], t32_start[i + 1] - t32_start[i], red);
    if (threadIdx.x == 0) {
        CgState c;
        c.rho = rho;
        c.rho0 = rho;
        c.stopped = 0;
        c.iters = 0;
        c.breakdown = 0;
        c.pad = 0;
        st[i] = c;
    }
}

// gamma = <p, A p> of instance blockIdx.x from the adjoint's partials; step decision
__global__ __launch_bounds__(256) void k_multi_gamma(const double *__restrict__ part, int64_t G,
                                                     const CgState *__restrict__ st,
                                                     CgStep *__restrict__ step, double rtol)
{
    __shared__ double red[256];
    const int i = blockIdx.x;
    const double gamma = sum_part_block(part + int64_t(i) * G, G, red);
    if (threadIdx.x == 0) {
        double a;
        CgStep o;
        o.stopped = cg_decide(st[i], gamma, rtol, &a);
        o.a = a;
        o.gamma = gamma;
        o.pad = 0;
        step[i] = o;
    }
}

// x += a p, r -= a q over the instance's vector blocks; partial <r, r> per block
template <class T>
__global__ __launch_bounds__(kVecThreads) void k_multi_xr(T *__restrict__ x, T *__restrict__ r,
                                                          const T *__restrict__ p,
                                                          const T *__restrict__ q,
                                                          const MultiInst *__restrict__ inst,
                                                          const int64_t *__restrict__ vb_start,
                                                          int count, const CgStep *__restrict__ step,
                                                          double *__restrict__ part)
{
    __shared__ double red[kVecThreads];
    const int i = find_inst(vb_start, count, blockIdx.x);
    const CgStep s = step[i];
    if (s.stopped) return;   // uniform per block; the partials are then unused
    const MultiInst &I = inst[i];
    const int64_t lb = int64_t(blockIdx.x) - vb_start[i], nbk = vb_start[i + 1] - vb_start[i];
    const T at = T(s.a);
    double acc = 0.0;
    for (int64_t e = lb * kVecThreads + threadIdx.x; e < I.nn; e += nbk * kVecThreads) {
        const int64_t j = I.img_off + e;
        x[j] = fma(at, p[j], x[j]);
        const T rn = fma(-at, q[j], r[j]);
        r[j] = rn;
        acc += double(rn) * double(rn);
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// rho' of instance blockIdx.x and the next state (ring slot (it+1) % 2)
__global__ __launch_bounds__(256) void k_multi_beta(const double *__restrict__ part,
                                                    const int64_t *__restrict__ vb_start,
                                                    const CgState *__restrict__ st,
                                                    const CgStep *__restrict__ step,
                                                    CgState *__restrict__ st_next, int it)
{
    __shared__ double red[256];
    const int i = blockIdx.x;
    const CgState c = st[i];
    const int stop = step[i].stopped;
    if (stop) {
        if (threadIdx.x == 0) {
            CgState o = c;
            o.stopped = 1;
            if (stop == 2 && !c.stopped) o.breakdown = it + 1;
            st_next[i] = o;
        }
        return;
    }
    const double rn = sum_part_block(part + vb_start[i], vb_start[i + 1] - vb_start[i], red);
    if (threadIdx.x == 0) {
        CgState o = c;
        o.rho = rn;
        o.iters = c.iters + 1;
        st_next[i] = o;
    }
}

// p = r + beta p (+ transposed copy) per 32x32 tile, beta = rho'/rho
template <class T>
__global__ __launch_bounds__(256) void k_multi_p(const T *__restrict__ r, T *__restrict__ p,
                                                 T *__restrict__ pT,
                                                 const MultiInst *__restrict__ inst,
                                                 const int64_t *__restrict__ t32_start, int count,
                                                 const CgState *__restrict__ st,
                                                 const CgState *__restrict__ st_next,
                                                 const CgStep *__restrict__ step)
{
    __shared__ T tile[32][33];
    const int i = find_inst(t32_start, count, blockIdx.x);
    if (step[i].stopped) return;
    const MultiInst &I = inst[i];
    const T beta = T(st_next[i].rho / st[i].rho);
    const int64_t t = int64_t(blockIdx.x) - t32_start[i];
    const int bx = int(t % I.tiles32) * 32, by = int(t / I.tiles32) * 32, n = I.n;
    const int64_t off = I.img_off;
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int iy = by + k, ix = bx + threadIdx.x;
        if (iy < n && ix < n) {
            const int64_t j = off + int64_t(iy) * n + ix;
            const T v = fma(beta, p[j], r[j]);
            p[j] = v;
            tile[k][threadIdx.x] = v;
        }
    }
    if (!pT || !I.need_T) return;
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int ix = bx + k, iy = by + threadIdx.x;
        if (ix < n && iy < n) pT[off + int64_t(ix) * n + iy] = tile[threadIdx.x][k];
    }
}

__global__ void k_multi_info(const CgState *__restrict__ st, radon_cg_info *__restrict__ info,
                             int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    radon_cg_info o;
    o.iterations = st[i].iters;
    o.breakdown = st[i].breakdown;
    o.rho0 = st[i].rho0;
    o.rho = st[i].rho;
    info[i] = o;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// waves per ray bundle of the group forward (the single-operator default)
constexpr int kMultiFwdWaves = 2;

static int64_t adj_grid(const Multi &m) { return m.n_grp < kPersistentBlocks ? m.n_grp : kPersistentBlocks; }
static int64_t fwd_grid(const Multi &m) { return m.n_fwork < kPersistentBlocks ? m.n_fwork : kPersistentBlocks; }

template <class T>
struct MultiBufs {
    uint32_t *tickets = nullptr;                   // [8 * kTicketStride] forward work counters
    T *xT = nullptr, *y = nullptr;                 // products
    T *fpart = nullptr;                            // band partials of the banded instances
    T *r = nullptr, *p = nullptr, *pT = nullptr, *q = nullptr;
    double *part_adj = nullptr, *part_t = nullptr, *part_vb = nullptr;
    CgState *st = nullptr;                         // [2][count]
    CgStep *step = nullptr;                        // [count]
};

template <class T>
static void carve_multi(const Multi &m, bool cg, Carver &c, MultiBufs<T> &w)
{
    const int64_t ni = m.img_off[size_t(m.count)], ns = m.sino_off[size_t(m.count)];
    w.tickets = c.take<uint32_t>(8 * kTicketStride);
    w.y = c.take<T>(ns);
    w.fpart = c.take<T>(m.n_fpart);
    if (!cg) {
        w.xT = m.any_T ? c.take<T>(ni) : nullptr;
        return;
    }
    w.r = c.take<T>(ni);
    w.p = c.take<T>(ni);
    w.pT = m.any_T ? c.take<T>(ni) : nullptr;
    w.q = c.take<T>(ni);
    w.part_adj = c.take<double>(int64_t(m.count) * adj_grid(m));
    w.part_t = c.take<double>(m.n_t32);
    w.part_vb = c.take<double>(m.n_vb);
    w.st = c.take<CgState>(2 * int64_t(m.count));
    w.step = c.take<CgStep>(m.count);
}

static int64_t multi_ws_bytes(const Multi &m, bool cg)
{
    Carver c(nullptr);
    if (m.vsize == 4) {
        MultiBufs<float> w;
        carve_multi(m, cg, c, w);
    } else {
        MultiBufs<double> w;
        carve_multi(m, cg, c, w);
    }
    return c.used;
}

template <class TM, class TV>
static int multi_launch_fwd(const Multi &m, const TV *x, const TV *xT, TV *y, TV *fpart,
                            uint32_t *tickets, hipStream_t s)
{
    k_ticket_reset<<<1, 64, 0, s>>>(tickets);
    SCT_TRY(check_launch("k_ticket_reset"));
    const unsigned g = unsigned(fwd_grid(m)), bs = 64 * kMultiFwdWaves;
    switch (m.bw) {
    case 64:
        k_multi_fwd<TM, TV, kMultiFwdWaves, 64><<<g, bs, 0, s>>>(m.fwork, m.n_fwork, m.inst, x,
                                                                 xT ? xT : x, y, fpart, tickets);
        break;
    case 32:
        k_multi_fwd<TM, TV, kMultiFwdWaves, 32><<<g, bs, 0, s>>>(m.fwork, m.n_fwork, m.inst, x,
                                                                 xT ? xT : x, y, fpart, tickets);
        break;
    default:
        k_multi_fwd<TM, TV, kMultiFwdWaves, 16><<<g, bs, 0, s>>>(m.fwork, m.n_fwork, m.inst, x,
                                                                 xT ? xT : x, y, fpart, tickets);
        break;
    }
    SCT_TRY(check_launch("k_multi_fwd"));
    // banded instances: their band partials into their sinograms
    for (int i = 0; i < m.count; ++i) {
        const Op &op = *m.ops[size_t(i)];
        if (m.part_off[size_t(i)] < 0) continue;
        k_fwd_band_sum<TV><<<dim3(unsigned((op.rows + 255) / 256), 1u), 256, 0, s>>>(
            op.fb, fpart + m.part_off[size_t(i)], y + m.sino_off[size_t(i)], op.rows, op.n_bins, op.bmap,
            op.n_bands, kBandLines);
        SCT_TRY(check_launch("k_fwd_band_sum"));
    }
    return RADON_OK;
}

template <class TM, class TV>
static int multi_launch_adj(const Multi &m, const TV *y, const TV *x, TV *out, int normal,
                            double *part, hipStream_t s)
{
    const unsigned g = unsigned(adj_grid(m));
    switch (m.adj_w) {
    case 4:
        k_multi_adj<TM, TV, 4><<<g, 256, 0, s>>>(m.grp_start, m.count, m.inst, y, x, out, normal, part);
        break;
    case 2:
        k_multi_adj<TM, TV, 2><<<g, 128, 0, s>>>(m.grp_start, m.count, m.inst, y, x, out, normal, part);
        break;
    default:
        k_multi_adj<TM, TV, 1><<<g, 64, 0, s>>>(m.grp_start, m.count, m.inst, y, x, out, normal, part);
        break;
    }
    return check_launch("k_multi_adj");
}

template <class TV>
static int multi_launch_transpose(const Multi &m, const TV *x, TV *xT, hipStream_t s)
{
    if (!m.any_T) return RADON_OK;
    k_multi_transpose<TV><<<unsigned(m.n_t32), dim3(32, 8), 0, s>>>(x, xT, m.inst, m.t32_start, m.count);
    return check_launch("k_multi_transpose");
}

template <class TM, class TV>
static int multi_products(const Multi &m, int which, const void *in, void *out_v, void *ws,
                          hipStream_t s)
{
    Carver c(ws);
    MultiBufs<TV> w;
    carve_multi(m, false, c, w);
    const TV *x = static_cast<const TV *>(in);
    TV *out = static_cast<TV *>(out_v);
    if (which == 0) {   // forward
        SCT_TRY(multi_launch_transpose<TV>(m, x, w.xT, s));
        return multi_launch_fwd<TM, TV>(m, x, w.xT, out, w.fpart, w.tickets, s);
    }
    if (which == 1)     // adjoint
        return multi_launch_adj<TM, TV>(m, x, nullptr, out, 0, nullptr, s);
    SCT_TRY(multi_launch_transpose<TV>(m, x, w.xT, s));   // normal operator
    SCT_TRY((multi_launch_fwd<TM, TV>(m, x, w.xT, w.y, w.fpart, w.tickets, s)));
    return multi_launch_adj<TM, TV>(m, w.y, x, out, 1, nullptr, s);
}

template <class TM, class TV>
static int multi_cg(const Multi &m, const void *rhs_v, void *x_v, int n_iter, double rtol, void *ws,
                    radon_cg_info *info, hipStream_t s)
{
    Carver c(ws);
    MultiBufs<TV> w;
    carve_multi(m, true, c, w);
    const TV *rhs = static_cast<const TV *>(rhs_v);
    TV *x = static_cast<TV *>(x_v);
    const int64_t ni = m.img_off[size_t(m.count)];
    const int vb = vec_blocks(ni);
    k_fill<TV><<<vb, kVecThreads, 0, s>>>(x, TV(0), ni);
    SCT_TRY(check_launch("k_fill"));
    k_copy<TV><<<vb, kVecThreads, 0, s>>>(rhs, w.r, ni);
    SCT_TRY(check_launch("k_copy"));
    k_multi_cg_start<TV><<<unsigned(m.n_t32), dim3(32, 8), 0, s>>>(w.r, w.p, w.pT, m.inst, m.t32_start,
                                                                  m.count, w.part_t);
    SCT_TRY(check_launch("k_multi_cg_start"));
    k_multi_begin<<<unsigned(m.count), 256, 0, s>>>(w.part_t, m.t32_start, w.st);
    SCT_TRY(check_launch("k_multi_begin"));
    for (int it = 0; it < n_iter; ++it) {
        CgState *cur = w.st + int64_t(it & 1) * m.count, *nxt = w.st + int64_t((it + 1) & 1) * m.count;
        SCT_TRY((multi_launch_fwd<TM, TV>(m, w.p, w.pT, w.y, w.fpart, w.tickets, s)));
        SCT_TRY((multi_launch_adj<TM, TV>(m, w.y, w.p, w.q, 1, w.part_adj, s)));
        k_multi_gamma<<<unsigned(m.count), 256, 0, s>>>(w.part_adj, adj_grid(m), cur, w.step, rtol);
        SCT_TRY(check_launch("k_multi_gamma"));
        k_multi_xr<TV><<<unsigned(m.n_vb), kVecThreads, 0, s>>>(x, w.r, w.p, w.q, m.inst, m.vb_start,
                                                               m.count, w.step, w.part_vb);
        SCT_TRY(check_launch("k_multi_xr"));
        k_multi_beta<<<unsigned(m.count), 256, 0, s>>>(w.part_vb, m.vb_start, cur, w.step, nxt, it);
        SCT_TRY(check_launch("k_multi_beta"));
        k_multi_p<TV><<<unsigned(m.n_t32), dim3(32, 8), 0, s>>>(w.r, w.p, w.pT, m.inst, m.t32_start,
                                                               m.count, cur, nxt, w.step);
        SCT_TRY(check_launch("k_multi_p"));
    }
    if (info) {
        k_multi_info<<<unsigned((m.count + 63) / 64), 64, 0, s>>>(
            w.st + int64_t(n_iter & 1) * m.count, info, m.count);
        SCT_TRY(check_launch("k_multi_info"));
    }
    return RADON_OK;
}

template <class F>
static int multi_dispatch(const Multi &m, F &&f)
{
    switch (m.dtype) {
    case SPARSECT_F32: return f(static_cast<float *>(nullptr), static_cast<float *>(nullptr));
    case SPARSECT_F64: return f(static_cast<double *>(nullptr), static_cast<double *>(nullptr));
    default: return f(static_cast<float *>(nullptr), static_cast<double *>(nullptr));
    }
}

static void free_multi(Multi *m)
{
    if (!m) return;
    for (void *p : m->owned) (void)hipFree(p);
    delete m;
}

static int multi_alloc(Multi &m, void **p, int64_t bytes)
{
    SCT_HIP(hipMalloc(p, size_t(bytes > 0 ? bytes : 1)));
    m.owned.push_back(*p);
    return RADON_OK;
}

// Host side of a group: instance descriptors, the concatenated forward work
// list and the instance start tables, before they go to the device.
struct MultiPlan {
    std::vector<MultiInst> hi;
    std::vector<int64_t> grp, t32, vbs;
    std::vector<int2> work;
};

// Bytes of the group's device tables, 256-byte aligned one after another.
static int64_t multi_table_bytes(const Multi &m)
{
    Carver c(nullptr);
    c.take<MultiInst>(m.count);
    c.take<int2>(m.n_fwork);
    for (int k = 0; k < 3; ++k) c.take<int64_t>(int64_t(m.count) + 1);
    return c.used;
}

// The tables into `tables` (caller storage of multi_table_bytes(m) bytes), or
// into allocations the handle owns when tables is NULL.
static int place_multi(Multi &m, const MultiPlan &pl, void *tables)
{
    if (tables) {
        Carver c(tables);
        m.inst = c.take<MultiInst>(m.count);
        m.fwork = c.take<int2>(m.n_fwork);
        m.grp_start = c.take<int64_t>(int64_t(m.count) + 1);
        m.t32_start = c.take<int64_t>(int64_t(m.count) + 1);
        m.vb_start = c.take<int64_t>(int64_t(m.count) + 1);
    } else {
        SCT_TRY(multi_alloc(m, reinterpret_cast<void **>(&m.inst), int64_t(sizeof(MultiInst)) * m.count));
        SCT_TRY(multi_alloc(m, reinterpret_cast<void **>(&m.fwork), int64_t(sizeof(int2)) * m.n_fwork));
        SCT_TRY(multi_alloc(m, reinterpret_cast<void **>(&m.grp_start), 8 * (int64_t(m.count) + 1)));
        SCT_TRY(multi_alloc(m, reinterpret_cast<void **>(&m.t32_start), 8 * (int64_t(m.count) + 1)));
        SCT_TRY(multi_alloc(m, reinterpret_cast<void **>(&m.vb_start), 8 * (int64_t(m.count) + 1)));
    }
    SCT_HIP(hipMemcpy(m.inst, pl.hi.data(), sizeof(MultiInst) * pl.hi.size(), hipMemcpyHostToDevice));
    SCT_HIP(hipMemcpy(m.fwork, pl.work.data(), sizeof(int2) * pl.work.size(), hipMemcpyHostToDevice));
    SCT_HIP(hipMemcpy(m.grp_start, pl.grp.data(), 8 * pl.grp.size(), hipMemcpyHostToDevice));
    SCT_HIP(hipMemcpy(m.t32_start, pl.t32.data(), 8 * pl.t32.size(), hipMemcpyHostToDevice));
    SCT_HIP(hipMemcpy(m.vb_start, pl.vbs.data(), 8 * pl.vbs.size(), hipMemcpyHostToDevice));
    return RADON_OK;
}

static int plan_multi(Multi &m, const radon_op *const *ops, int count, const double *alpha,
                      const double *lambda, const double *sigma, MultiPlan &pl)
{
    m.count = count;
    m.dtype = as_op(ops[0])->dtype;
    m.vsize = as_op(ops[0])->vsize;
    std::vector<MultiInst> &hi = pl.hi;
    std::vector<int64_t> &grp = pl.grp, &t32 = pl.t32, &vbs = pl.vbs;
    std::vector<int2> &work = pl.work;
    hi.assign(static_cast<size_t>(count), MultiInst{});
    grp.assign(size_t(count) + 1, 0);
    t32.assign(size_t(count) + 1, 0);
    vbs.assign(size_t(count) + 1, 0);
    work.clear();
    m.img_off.assign(size_t(count) + 1, 0);
    m.sino_off.assign(size_t(count) + 1, 0);
    m.part_off.assign(size_t(count), -1);
    int64_t meas_sum = 0;
    for (int i = 0; i < count; ++i) {
        const Op &op = *as_op(ops[i]);
        m.ops.push_back(&op);
        MultiInst &I = hi[size_t(i)];
        I.fb = op.fb;
        I.f_idx = op.f_idx;
        I.f_v0 = op.f_v0;
        I.f_v1 = op.f_v1;
        I.f_edge = op.f_edge;
        I.a_rel = op.a_rel;
        I.a_base = op.a_base;
        I.a_v0 = op.a_v0;
        I.a_v1 = op.a_v1;
        I.n_ag = op.n_ag;
        I.nn = op.nn;
        I.rows = op.rows;
        I.img_off = m.img_off[size_t(i)];
        I.sino_off = m.sino_off[size_t(i)];
        I.alpha = alpha ? alpha[i] : 1.0;
        I.lambda = lambda ? lambda[i] : 0.0;
        I.sigma = sigma ? sigma[i] : 0.0;
        I.n = op.n;
        I.n_meas = op.n_meas;
        I.n_aq = op.n_aq;
        I.nb = op.n_bins;
        I.tiles8 = op.tiles;
        I.tiles32 = tiles_of(op.n);
        I.need_T = op.need_T ? 1 : 0;
        // banded forward for instances that have bands and fit the packed
        // (band << 24 | bundle) entries
        const bool banded = op.n_bands > 0 && op.n_bands < 128 && op.n_fb < (int64_t(1) << 24);
        I.n_bands = banded ? op.n_bands : 0;
        I.part_off = banded ? m.n_fpart : 0;
        m.part_off[size_t(i)] = banded ? m.n_fpart : -1;
        if (banded) {
            const int64_t al = 256 / m.vsize;
            m.n_fpart += (int64_t(op.n_bands) * op.rows + al - 1) / al * al;
        }
        m.any_T = m.any_T || op.need_T;
        meas_sum += op.n_meas;
        // offsets: 256-byte aligned starts keep every instance's loads aligned
        const int64_t al = 256 / m.vsize;
        m.img_off[size_t(i) + 1] = I.img_off + (op.nn + al - 1) / al * al;
        m.sino_off[size_t(i) + 1] = I.sino_off + (op.rows + al - 1) / al * al;
        grp[size_t(i) + 1] = grp[size_t(i)] + op.n_ag;
        t32[size_t(i) + 1] = t32[size_t(i)] + int64_t(I.tiles32) * I.tiles32;
        vbs[size_t(i) + 1] = vbs[size_t(i)] + vec_blocks(op.nn);
        if (banded) {
            std::vector<int2> border(size_t(op.n_band_order));
            SCT_HIP(hipMemcpy(border.data(), op.fb_band_order, 8 * size_t(op.n_band_order),
                              hipMemcpyDeviceToHost));
            for (const int2 &e : border) work.push_back(make_int2(i, e.x < 0 ? -1 : (e.y << 24) | e.x));
        } else {
            std::vector<int32_t> order(size_t(op.n_order));
            SCT_HIP(hipMemcpy(order.data(), op.fb_order, 4 * size_t(op.n_order), hipMemcpyDeviceToHost));
            for (int32_t b : order) work.push_back(make_int2(i, b));
        }
        while (work.size() % 8) work.push_back(make_int2(i, -1));
    }
    m.n_grp = grp[size_t(count)];
    m.n_t32 = t32[size_t(count)];
    m.n_vb = vbs[size_t(count)];
    m.n_fwork = int64_t(work.size());
    if (m.n_t32 > 0x7fffffffLL || m.n_vb > 0x7fffffffLL)
        return set_error(RADON_EUNSUPPORTED, "too many vector tiles in one group");
    // the single-operator rule applied to the mean measured-angle count
    m.adj_w = adj_waves_for(int(meas_sum / count));
    return RADON_OK;
}

static int check_multi(const radon_multi *p)
{
    if (!p) return set_error(RADON_EINVAL, "multi handle is NULL");
    return RADON_OK;
}

inline const Multi *as_multi(const radon_multi *p) { return reinterpret_cast<const Multi *>(p); }

}  // namespace sct

using namespace sct;

static int check_group_ops(const radon_op *const *ops, int32_t count)
{
    if (!ops) return set_error(RADON_EINVAL, "ops is NULL");
    if (count < 1 || count > 65535) return set_error(RADON_EINVAL, "count must be in [1, 65535] (got %d)", count);
    for (int i = 0; i < count; ++i) {
        SCT_TRY(check_op(ops[i]));
        if (as_op(ops[i])->dtype != as_op(ops[0])->dtype)
            return set_error(RADON_EINVAL, "operator %d has another dtype than operator 0", i);
        if (as_op(ops[i])->bw != as_op(ops[0])->bw)
            return set_error(RADON_EINVAL, "operator %d has another forward bundle width than operator 0", i);
        if (as_op(ops[i])->sym)
            return set_error(RADON_EUNSUPPORTED, "operator %d is stored by symmetry, which a group does not take", i);
    }
    return RADON_OK;
}

// Plans the group and places its tables (into `tables` when given).
static int create_group(const radon_op *const *ops, int32_t count, const double *alpha,
                        const double *lambda, const double *sigma, void *tables, int64_t tables_bytes,
                        radon_multi **out)
{
    Multi *m = new (std::nothrow) Multi;
    if (!m) return set_error(RADON_EINVAL, "out of host memory");
    m->bw = as_op(ops[0])->bw;
    MultiPlan pl;
    int rc = plan_multi(*m, ops, count, alpha, lambda, sigma, pl);
    if (rc == RADON_OK && tables && tables_bytes < multi_table_bytes(*m))
        rc = set_error(RADON_EWORKSPACE, "the tables need %lld bytes, %lld given",
                       (long long)multi_table_bytes(*m), (long long)tables_bytes);
    if (rc == RADON_OK) rc = place_multi(*m, pl, tables);
    if (rc != RADON_OK) {
        free_multi(m);
        return rc;
    }
    *out = reinterpret_cast<radon_multi *>(m);
    return RADON_OK;
}

extern "C" int radon_multi_create(const radon_op *const *ops, int32_t count, const double *alpha,
                                  const double *lambda, const double *sigma, radon_multi **out)
{
    clear_error();
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    *out = nullptr;
    SCT_TRY(check_group_ops(ops, count));
    return create_group(ops, count, alpha, lambda, sigma, nullptr, 0, out);
}

extern "C" int radon_multi_table_bytes(const radon_op *const *ops, int32_t count, int64_t *bytes)
{
    clear_error();
    if (!bytes) return set_error(RADON_EINVAL, "bytes is NULL");
    *bytes = 0;
    SCT_TRY(check_group_ops(ops, count));
    Multi m;
    m.bw = as_op(ops[0])->bw;
    MultiPlan pl;
    SCT_TRY(plan_multi(m, ops, count, nullptr, nullptr, nullptr, pl));
    *bytes = multi_table_bytes(m);
    return RADON_OK;
}

extern "C" int radon_multi_create_into(const radon_op *const *ops, int32_t count, const double *alpha,
                                       const double *lambda, const double *sigma, void *tables,
                                       int64_t tables_bytes, radon_multi **out)
{
    clear_error();
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    *out = nullptr;
    if (!tables) return set_error(RADON_EINVAL, "tables is NULL");
    if (reinterpret_cast<uintptr_t>(tables) & 255) return set_error(RADON_EINVAL, "tables must be 256-byte aligned");
    SCT_TRY(check_group_ops(ops, count));
    return create_group(ops, count, alpha, lambda, sigma, tables, tables_bytes, out);
}

extern "C" void radon_multi_destroy(radon_multi *p) { free_multi(reinterpret_cast<Multi *>(p)); }

extern "C" int radon_multi_info(const radon_multi *p, int64_t *img_off, int64_t *sino_off,
                                int64_t *ws_products, int64_t *ws_cg, int32_t *fwd_waves,
                                int32_t *adj_waves)
{
    clear_error();
    SCT_TRY(check_multi(p));
    const Multi &m = *as_multi(p);
    for (int i = 0; i <= m.count; ++i) {
        if (img_off) img_off[i] = m.img_off[size_t(i)];
        if (sino_off) sino_off[i] = m.sino_off[size_t(i)];
    }
    if (ws_products) *ws_products = multi_ws_bytes(m, false);
    if (ws_cg) *ws_cg = multi_ws_bytes(m, true);
    if (fwd_waves) *fwd_waves = kMultiFwdWaves;
    if (adj_waves) *adj_waves = m.adj_w;
    return RADON_OK;
}

extern "C" int radon_multi_apply(const radon_multi *p, int32_t which, const void *in, void *out,
                                 void *ws, int64_t ws_bytes, void *stream)
{
    clear_error();
    SCT_TRY(check_multi(p));
    if (which < 0 || which > 2) return set_error(RADON_EINVAL, "which must be 0, 1 or 2 (got %d)", which);
    if (!in || !out) return set_error(RADON_EINVAL, "in and out must be non-NULL");
    if (in == out) return set_error(RADON_EINVAL, "out must not alias in");
    const Multi &m = *as_multi(p);
    SCT_TRY(check_ws(ws, ws_bytes, multi_ws_bytes(m, false), "radon_multi_apply"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    return multi_dispatch(m, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        return multi_products<TM, TV>(m, which, in, out, ws, s);
    });
}

extern "C" int radon_multi_cg(const radon_multi *p, const void *rhs, void *x, int32_t n_iter,
                              double rtol, void *ws, int64_t ws_bytes, radon_cg_info *info,
                              void *stream)
{
    clear_error();
    SCT_TRY(check_multi(p));
    if (!rhs || !x) return set_error(RADON_EINVAL, "rhs and x must be non-NULL");
    if (rhs == x) return set_error(RADON_EINVAL, "x must not alias rhs");
    if (n_iter < 0) return set_error(RADON_EINVAL, "n_iter must be >= 0 (got %d)", n_iter);
    if (!(rtol >= 0.0)) return set_error(RADON_EINVAL, "rtol must be >= 0");
    const Multi &m = *as_multi(p);
    SCT_TRY(check_ws(ws, ws_bytes, multi_ws_bytes(m, true), "radon_multi_cg"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    return multi_dispatch(m, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        return multi_cg<TM, TV>(m, rhs, x, n_iter, rtol, ws, info, s);
    });
}

namespace sct {
// Record body(stream) on a private non-blocking stream of default priority and
// instantiate it as a radon_graph.
int capture_graph(const std::function<int(hipStream_t)> &body, radon_graph **out)
{
    hipStream_t cs = nullptr;
    SCT_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return set_error(RADON_EHIP, "hipStreamBeginCapture failed: %s", hipGetErrorString(e));
    }
    const int rc = body(cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc != RADON_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return set_error(RADON_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    Graph *G = new (std::nothrow) Graph;
    if (!G) {
        (void)hipGraphDestroy(g);
        return set_error(RADON_EINVAL, "out of host memory");
    }
    G->graph = g;
    e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete G;
        return set_error(RADON_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    *out = reinterpret_cast<radon_graph *>(G);
    return RADON_OK;
}
}  // namespace sct

extern "C" int radon_multi_cg_graph(const radon_multi *p, const void *rhs, void *x, int32_t n_iter,
                                    double rtol, void *ws, int64_t ws_bytes, radon_cg_info *info,
                                    radon_graph **out)
{
    clear_error();
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    *out = nullptr;
    SCT_TRY(check_multi(p));
    if (!rhs || !x) return set_error(RADON_EINVAL, "rhs and x must be non-NULL");
    if (rhs == x) return set_error(RADON_EINVAL, "x must not alias rhs");
    if (n_iter < 0) return set_error(RADON_EINVAL, "n_iter must be >= 0 (got %d)", n_iter);
    if (!(rtol >= 0.0)) return set_error(RADON_EINVAL, "rtol must be >= 0");
    const Multi &m = *as_multi(p);
    SCT_TRY(check_ws(ws, ws_bytes, multi_ws_bytes(m, true), "radon_multi_cg_graph"));
    return capture_graph(
        [&](hipStream_t cs) {
            return multi_dispatch(m, [&](auto *tm, auto *tv) {
                SCT_TYPES(tm, tv);
                return multi_cg<TM, TV>(m, rhs, x, n_iter, rtol, ws, info, cs);
            });
        },
        out);
}

extern "C" int radon_graph_launch(const radon_graph *p, void *stream)
{
    clear_error();
    if (!p) return set_error(RADON_EINVAL, "graph is NULL");
    const Graph *G = reinterpret_cast<const Graph *>(p);
    SCT_HIP(hipGraphLaunch(G->exec, static_cast<hipStream_t>(stream)));
    return RADON_OK;
}

extern "C" void radon_graph_destroy(radon_graph *p)
{
    if (!p) return;
    Graph *G = reinterpret_cast<Graph *>(p);
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
}
