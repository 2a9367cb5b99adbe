// Operator construction: Siddon ray tracing on the GPU, the CSR of MR, and the
// two slotted layouts the apply kernels stream (Section 3 of the paper: the
// sparse operator is precomputed once for a fixed geometry).
//
// This file is compiled with FP contraction off so that every crossing
// parameter and length is computed with the plain IEEE operations of its
// formula.
#include "internal.hpp"

#include <hipcub/hipcub.hpp>

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

namespace sct {

static thread_local std::string g_err;

int set_error(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }

static const char *last_error() { return g_err.c_str(); }

int check_op(const radon_op *p)
{
    if (!p) return set_error(RADON_EINVAL, "operator handle is NULL");
    const Op *op = as_op(p);
    if (op->n <= 0 || !op->fb || !op->a_v0 || !op->a_rel) return set_error(RADON_ESTATE, "operator handle is not built");
    return RADON_OK;
}

int check_batch(int32_t batch)
{
    if (batch < 1) return set_error(RADON_EINVAL, "batch must be >= 1 (got %d)", batch);
    return RADON_OK;
}

int check_ws(const void *ws, int64_t ws_bytes, int64_t need, const char *what)
{
    if (need > 0 && (!ws || ws_bytes < need))
        return set_error(RADON_EWORKSPACE, "%s needs a workspace of %lld bytes (got %lld%s)", what,
                         (long long)need, (long long)ws_bytes, ws ? "" : ", NULL pointer");
    return RADON_OK;
}

// cos/sin of pi*k/na reduced to [0, pi/4]: 0, pi/4 and pi/2 come out exact,
// theta and pi - theta get cosines of opposite sign and equal magnitude, and
// angles symmetric about pi/4 swap cos and sin exactly.
static void angle_cos_sin(int k, int na, double *c, double *s)
{
    int kk = k;
    bool negate = false;
    if (2 * kk > na) {
        kk = na - kk;
        negate = true;
    }
    if (kk == 0) {
        *c = 1.0;
        *s = 0.0;
    } else if (2 * kk == na) {
        *c = 0.0;
        *s = 1.0;
    } else if (4 * kk == na) {
        *c = std::sqrt(0.5);
        *s = std::sqrt(0.5);
    } else if (4 * kk > na) {
        const double comp = M_PI * double(na - 2 * kk) / (2.0 * double(na));
        *c = std::sin(comp);
        *s = std::cos(comp);
    } else {
        const double th = M_PI * double(kk) / double(na);
        *c = std::cos(th);
        *s = std::sin(th);
    }
    if (negate) *c = -*c;
}

// ---------------------------------------------------------------------------
// Ray tracing
// ---------------------------------------------------------------------------

constexpr double kSliver = 1e-12;

// Visits the pixels of ray {p . (c, s) = sb} in the order the parametrisation
// p(t) = sb (c, s) + t (-s, c) meets them, calling emit(j, length) once per
// pixel (a segment split only by a dropped sliver is merged back).
template <class Emit>
__device__ void trace_ray(int n, double c, double s, double sb, Emit &&emit)
{
    const double h = 0.5 * double(n);
    if (s == 0.0 || c == 0.0) {
        // Axis-aligned: theta = 0 is the vertical line x = sb (t runs up y),
        // theta = pi/2 the horizontal line y = sb (t runs down x).
        const bool vertical = (s == 0.0);
        const double pos = (vertical ? sb * c : sb * s) + h;
        if (pos == floor(pos)) {
            if (pos < 0.0 || pos > double(n)) return;
            const int e = int(pos);   // edge between pixel lines e-1 and e
            if (vertical) {
                for (int iy = 0; iy < n; ++iy) {
                    if (e - 1 >= 0) emit(iy * n + e - 1, 0.5);
                    if (e < n) emit(iy * n + e, 0.5);
                }
            } else {
                for (int ix = n - 1; ix >= 0; --ix) {
                    if (e - 1 >= 0) emit((e - 1) * n + ix, 0.5);
                    if (e < n) emit(e * n + ix, 0.5);
                }
            }
            return;
        }
        if (!(pos > 0.0 && pos < double(n))) return;
        const int q = int(floor(pos));
        if (vertical) {
            for (int iy = 0; iy < n; ++iy) emit(iy * n + q, 1.0);
        } else {
            for (int ix = n - 1; ix >= 0; --ix) emit(q * n + ix, 1.0);
        }
        return;
    }

    const double sc = sb * c, ss = sb * s;
    const double tx0 = (sc - (-h)) / s, tx1 = (sc - h) / s;
    const double ty0 = ((-h) - ss) / c, ty1 = (h - ss) / c;
    const double tin = fmax(fmin(tx0, tx1), fmin(ty0, ty1));
    const double tout = fmin(fmax(tx0, tx1), fmax(ty0, ty1));
    if (!(tout - tin > kSliver)) return;
    const double INF = __builtin_huge_val();

    // vertical lines x = q - h meet the ray at increasing t for decreasing q (s > 0)
    int qx = n - 1;
    auto next_x = [&]() -> double {
        while (qx >= 1) {
            const double X = double(qx) - h;
            const double t = (sc - X) / s;
            --qx;
            if (t > tin) return t < tout ? t : INF;
        }
        return INF;
    };
    // horizontal lines y = q - h: increasing t for increasing q when c > 0
    const int dq = c > 0.0 ? 1 : -1;
    int qy = c > 0.0 ? 1 : n - 1;
    auto next_y = [&]() -> double {
        while (qy >= 1 && qy <= n - 1) {
            const double Y = double(qy) - h;
            const double t = (Y - ss) / c;
            qy += dq;
            if (t > tin) return t < tout ? t : INF;
        }
        return INF;
    };

    int lastj = -1;
    double acc = 0.0;
    double tx = next_x(), ty = next_y(), tcur = tin;
    for (;;) {
        double tn = fmin(tx, ty);
        const bool end = !(tn < tout);
        if (end) tn = tout;
        const double len = tn - tcur;
        if (len > kSliver) {
            const double tm = 0.5 * (tcur + tn);
            const double px = sc - tm * s, py = ss + tm * c;
            int ix = int(floor(px + h)), iy = int(floor(py + h));
            ix = ix < 0 ? 0 : (ix > n - 1 ? n - 1 : ix);
            iy = iy < 0 ? 0 : (iy > n - 1 ? n - 1 : iy);
            const int j = iy * n + ix;
            if (j == lastj) {
                acc += len;
            } else {
                if (lastj >= 0) emit(lastj, acc);
                lastj = j;
                acc = len;
            }
        }
        if (end) break;
        if (tx <= ty) tx = next_x();
        else ty = next_y();
        tcur = tn;
    }
    if (lastj >= 0) emit(lastj, acc);
}

__device__ inline bool is_horiz(double c, double s) { return fabs(s) > fabs(c); }

// Pass 1: entries per measured ray and the range of major lines it covers.
__global__ void k_ray_count(const double2 *__restrict__ cs, int n, int nb, int64_t rows,
                            int64_t *__restrict__ cnt, int32_t *__restrict__ mlo,
                            int32_t *__restrict__ mhi)
{
    const int64_t ray = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ray >= rows) return;
    const int a = int(ray / nb), b = int(ray % nb);
    const double c = cs[a].x, s = cs[a].y;
    const double sb = double(b) - 0.5 * double(nb - 1);
    const bool hz = is_horiz(c, s);
    int64_t count = 0;
    int lo = INT_MAX, hi = -1;
    trace_ray(n, c, s, sb, [&](int j, double) {
        ++count;
        const int m = hz ? j % n : j / n;
        lo = m < lo ? m : lo;
        hi = m > hi ? m : hi;
    });
    cnt[ray] = count;
    mlo[ray] = lo;
    mhi[ray] = hi;
}

// Bundle extents: union of the major ranges of up to 16 adjacent rays.
__global__ void k_bundle_span(const double2 *__restrict__ cs, const int32_t *__restrict__ mlo,
                              const int32_t *__restrict__ mhi, int nb, int nbpa, int64_t n_fb,
                              FwdBundle *__restrict__ fb, int64_t *__restrict__ slots)
{
    const int64_t B = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (B >= n_fb) return;
    const int a = int(B / nbpa), t = int(B % nbpa);
    const int ray0 = a * nb + t * kFwdLanes;
    const int nrays = min(kFwdLanes, nb - t * kFwdLanes);
    int lo = INT_MAX, hi = -1;
    for (int r = 0; r < nrays; ++r) {
        if (mhi[ray0 + r] >= 0) {
            lo = min(lo, mlo[ray0 + r]);
            hi = max(hi, mhi[ray0 + r]);
        }
    }
    FwdBundle d;
    d.off = 0;
    d.m0 = hi >= 0 ? lo : 0;
    d.nrows = hi >= 0 ? ((hi - lo + 1 + 3) / 4) * 4 : 0;
    d.ray0 = ray0;
    d.nrays = nrays;
    d.horiz = is_horiz(cs[a].x, cs[a].y) ? 1 : 0;
    d.pad = 0;
    fb[B] = d;
    slots[B] = int64_t(d.nrows) * kFwdLanes;
}

__global__ void k_bundle_off(FwdBundle *__restrict__ fb, const int64_t *__restrict__ incl,
                             int64_t n_fb)
{
    const int64_t B = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (B >= n_fb) return;
    fb[B].off = incl[B] - int64_t(fb[B].nrows) * kFwdLanes;
}

// Pass 2: write the CSR row and the ray's forward slots, and mark the first
// bin of every (pixel, angle) pair the ray touches.
template <class T>
__global__ void k_ray_fill(const double2 *__restrict__ cs, int n, int nb, int nbpa, int64_t rows,
                           int n_aq, int tiles, const int64_t *__restrict__ rp, int32_t *__restrict__ col,
                           T *__restrict__ val, const FwdBundle *__restrict__ fb,
                           uint16_t *__restrict__ f_idx, T *__restrict__ f_v0,
                           T *__restrict__ f_v1, int32_t *__restrict__ bin_tmp,
                           int32_t *__restrict__ bad)
{
    const int64_t ray = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ray >= rows) return;
    const int a = int(ray / nb), b = int(ray % nb);
    const double c = cs[a].x, s = cs[a].y;
    const double sb = double(b) - 0.5 * double(nb - 1);
    const bool hz = is_horiz(c, s);
    const FwdBundle d = fb[int64_t(a) * nbpa + b / kFwdLanes];
    const int r = b % kFwdLanes;
    int64_t o = rp[ray];
    int cur = -1, nline = 0, q0 = 0, q1 = 0;
    T w0 = T(0), w1 = T(0);
    const int64_t oend = rp[ray + 1];
    auto flush = [&]() {
        if (cur < 0) return;
        if (cur < d.m0 || cur >= d.m0 + d.nrows) {
            atomicOr(bad, 16);
            return;
        }
        const int64_t slot = fwd_slot(d.off, cur - d.m0, r);
        if (nline == 1) {
            f_idx[slot] = uint16_t(q0);
            f_v0[slot] = w0;
            f_v1[slot] = T(0);
        } else {
            if (q1 != q0 + 1 && q0 != q1 + 1) atomicOr(bad, 1);
            const bool first0 = q0 < q1;
            f_idx[slot] = uint16_t(first0 ? q0 : q1);
            f_v0[slot] = first0 ? w0 : w1;
            f_v1[slot] = first0 ? w1 : w0;
        }
    };
    trace_ray(n, c, s, sb, [&](int j, double len) {
        const T v = T(len);
        if (o < oend) {
            col[o] = j;
            val[o] = v;
        } else {
            atomicOr(bad, 4);
        }
        ++o;
        const int m = hz ? j % n : j / n;
        const int q = hz ? j / n : j % n;
        if (m != cur) {
            flush();
            cur = m;
            nline = 1;
            q0 = q;
            w0 = v;
        } else {
            if (nline >= 2) atomicOr(bad, 2);
            nline = 2;
            q1 = q;
            w1 = v;
        }
        atomicMin(&bin_tmp[adj_slot(j / n, j % n, a, n_aq, tiles)], b);
    });
    flush();
    if (o != oend) atomicOr(bad, 4);
}

// Pass 3: place each entry in its (pixel, angle) slot as the first or second bin.
template <class T>
__global__ void k_adj_fill(int n, int nb, int64_t rows, int n_aq, int tiles, const int64_t *__restrict__ rp,
                           const int32_t *__restrict__ col, const T *__restrict__ val,
                           const int32_t *__restrict__ bin_tmp, T *__restrict__ a_v0,
                           T *__restrict__ a_v1, int32_t *__restrict__ bad)
{
    const int64_t ray = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ray >= rows) return;
    const int a = int(ray / nb), b = int(ray % nb);
    for (int64_t e = rp[ray]; e < rp[ray + 1]; ++e) {
        const int j = col[e];
        const int64_t as = adj_slot(j / n, j % n, a, n_aq, tiles);
        const int first = bin_tmp[as];
        if (b == first) a_v0[as] = val[e];
        else if (b == first + 1) a_v1[as] = val[e];
        else atomicOr(bad, 8);
    }
}

// Per (tile, angle): the lowest first-bin over the tile's pixels.
__global__ void k_adj_base(const int32_t *__restrict__ bin_tmp, uint16_t *__restrict__ a_base,
                           int64_t n_ag, int n_aq)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;   // (tile, angle)
    if (i >= n_ag * n_aq * 4) return;
    const int64_t g = i / (int64_t(n_aq) * 4);
    const int a = int(i % (int64_t(n_aq) * 4));
    int lo = 65536;
    for (int l = 0; l < kAdjLanes; ++l) {
        const int t = bin_tmp[(((g * n_aq + (a >> 2)) * kAdjLanes + l) << 2) + (a & 3)];
        lo = t < lo ? t : lo;
    }
    a_base[i] = lo >= 65536 ? uint16_t(0) : uint16_t(lo);
}

__global__ void k_adj_finish(const int32_t *__restrict__ bin_tmp, const uint16_t *__restrict__ a_base,
                             uint8_t *__restrict__ a_rel, int64_t a_slots, int32_t *__restrict__ bad)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a_slots) return;
    // slot i = ((g*nq + aq)*64 + l)*4 + k  ->  base index (g*nq + aq)*4 + k
    const int64_t bi = ((i >> 2) / kAdjLanes) * 4 + (i & 3);
    const int t = bin_tmp[i];
    if (t >= 65536) {
        a_rel[i] = 0;
        return;
    }
    const int rel = t - int(a_base[bi]);
    if (rel < 0 || rel + 1 >= kAdjBand) atomicOr(bad, 32);
    a_rel[i] = uint8_t(rel < 0 ? 0 : (rel > kAdjBand - 2 ? kAdjBand - 2 : rel));
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static int grid_for(int64_t count, int block, unsigned *grid)
{
    const int64_t g = (count + block - 1) / block;
    if (g > int64_t(INT_MAX)) return set_error(RADON_EOVERFLOW, "grid too large");
    *grid = unsigned(g < 1 ? 1 : g);
    return RADON_OK;
}

static int op_alloc(Op &op, void **p, int64_t bytes)
{
    *p = nullptr;
    if (bytes <= 0) bytes = 256;
    SCT_HIP(hipMalloc(p, size_t(bytes)));
    op.owned.push_back(*p);
    op.device_bytes += bytes;
    return RADON_OK;
}

struct TempBufs {
    std::vector<void *> ptrs;
    ~TempBufs()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    int alloc(void **p, int64_t bytes)
    {
        *p = nullptr;
        if (bytes <= 0) bytes = 256;
        SCT_HIP(hipMalloc(p, size_t(bytes)));
        ptrs.push_back(*p);
        return RADON_OK;
    }
};

static void op_free(Op *op)
{
    if (!op) return;
    for (void *p : op->owned) (void)hipFree(p);
    delete op;
}

template <class T>
static int build_typed(Op &op, const std::vector<double> &cs_host, hipStream_t st)
{
    TempBufs tmp;
    const int n = op.n, nb = op.n_bins;
    const int64_t rows = op.rows;
    const int blk = 128;
    unsigned g;

    double2 *cs = nullptr;
    SCT_TRY(tmp.alloc(reinterpret_cast<void **>(&cs), int64_t(sizeof(double2)) * op.n_meas));
    SCT_HIP(hipMemcpyAsync(cs, cs_host.data(), sizeof(double2) * op.n_meas, hipMemcpyHostToDevice, st));

    int64_t *cnt = nullptr;
    int32_t *mlo = nullptr, *mhi = nullptr, *bad = nullptr;
    SCT_TRY(tmp.alloc(reinterpret_cast<void **>(&cnt), 8 * rows));
    SCT_TRY(tmp.alloc(reinterpret_cast<void **>(&mlo), 4 * rows));
    SCT_TRY(tmp.alloc(reinterpret_cast<void **>(&mhi), 4 * rows));
    SCT_TRY(tmp.alloc(reinterpret_cast<void **>(&bad), 4));
    SCT_HIP(hipMemsetAsync(bad, 0, 4, st));

    SCT_TRY(grid_for(rows, blk, &g));
    k_ray_count<<<g, blk, 0, st>>>(cs, n, nb, rows, cnt, mlo, mhi);
    SCT_TRY(check_launch("k_ray_count"));

    // row pointers
    SCT_TRY(op_alloc(op, reinterpret_cast<void **>(&op.rp), 8 * (rows + 1)));
    SCT_HIP(hipMemsetAsync(op.rp, 0, 8, st));
    size_t scan_bytes = 0, scan_bytes2 = 0;
    SCT_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, scan_bytes, cnt, op.rp + 1, rows, st));

    // bundles
    const int nbpa = (nb + kFwdLanes - 1) / kFwdLanes;
    op.n_fb = int64_t(op.n_meas) * nbpa;
    SCT_TRY(op_alloc(op, reinterpret_cast<void **>(&op.fb), int64_t(sizeof(FwdBundle)) * op.n_fb));
    int64_t *bslots = nullptr, *bincl = nullptr;
    SCT_TRY(tmp.alloc(reinterpret_cast<void **>(&bslots), 8 * op.n_fb));
    SCT_TRY(tmp.alloc(reinterpret_cast<void **>(&bincl), 8 * op.n_fb));
    SCT_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, scan_bytes2, bslots, bincl, op.n_fb, st));
    void *scan_tmp = nullptr;
    SCT_TRY(tmp.alloc(&scan_tmp, int64_t(scan_bytes > scan_bytes2 ? scan_bytes : scan_bytes2)));

    SCT_HIP(hipcub::DeviceScan::InclusiveSum(scan_tmp, scan_bytes, cnt, op.rp + 1, rows, st));
    SCT_TRY(grid_for(op.n_fb, blk, &g));
    k_bundle_span<<<g, blk, 0, st>>>(cs, mlo, mhi, nb, nbpa, op.n_fb, op.fb, bslots);
    SCT_TRY(check_launch("k_bundle_span"));
    size_t sb2 = scan_bytes2;
    SCT_HIP(hipcub::DeviceScan::InclusiveSum(scan_tmp, sb2, bslots, bincl, op.n_fb, st));
    k_bundle_off<<<g, blk, 0, st>>>(op.fb, bincl, op.n_fb);
    SCT_TRY(check_launch("k_bundle_off"));

    int64_t nnz = 0, fslots = 0;
    SCT_HIP(hipMemcpyAsync(&nnz, op.rp + rows, 8, hipMemcpyDeviceToHost, st));
    SCT_HIP(hipMemcpyAsync(&fslots, bincl + (op.n_fb - 1), 8, hipMemcpyDeviceToHost, st));
    SCT_HIP(hipStreamSynchronize(st));
    op.nnz = nnz;
    op.f_slots = fslots;
    if (nnz >= (int64_t(1) << 40)) return set_error(RADON_EOVERFLOW, "nnz %lld too large", (long long)nnz);

    const int64_t es = sizeof(T);
    SCT_TRY(op_alloc(op, reinterpret_cast<void **>(&op.col), 4 * nnz));
    SCT_TRY(op_alloc(op, &op.val, es * nnz));
    SCT_TRY(op_alloc(op, reinterpret_cast<void **>(&op.f_idx), 2 * fslots));
    SCT_TRY(op_alloc(op, &op.f_v0, es * fslots));
    SCT_TRY(op_alloc(op, &op.f_v1, es * fslots));
    SCT_HIP(hipMemsetAsync(op.f_idx, 0, size_t(2 * fslots), st));
    SCT_HIP(hipMemsetAsync(op.f_v0, 0, size_t(es * fslots), st));
    SCT_HIP(hipMemsetAsync(op.f_v1, 0, size_t(es * fslots), st));

    op.tiles = (op.n + 7) / 8;
    op.n_ag = int64_t(op.tiles) * op.tiles;
    op.n_aq = (op.n_meas + 3) / 4;
    op.a_slots = op.n_ag * kAdjLanes * 4 * op.n_aq;
    SCT_TRY(op_alloc(op, reinterpret_cast<void **>(&op.a_rel), op.a_slots));
    SCT_TRY(op_alloc(op, reinterpret_cast<void **>(&op.a_base), 2 * op.n_ag * op.n_aq * 4));
    SCT_TRY(op_alloc(op, &op.a_v0, es * op.a_slots));
    SCT_TRY(op_alloc(op, &op.a_v1, es * op.a_slots));
    SCT_HIP(hipMemsetAsync(op.a_v0, 0, size_t(es * op.a_slots), st));
    SCT_HIP(hipMemsetAsync(op.a_v1, 0, size_t(es * op.a_slots), st));
    int32_t *bin_tmp = nullptr;
    SCT_TRY(tmp.alloc(reinterpret_cast<void **>(&bin_tmp), 4 * op.a_slots));
    SCT_HIP(hipMemsetAsync(bin_tmp, 0x7f, size_t(4 * op.a_slots), st));   // 0x7f7f7f7f > any bin

    SCT_TRY(grid_for(rows, blk, &g));
    k_ray_fill<T><<<g, blk, 0, st>>>(cs, n, nb, nbpa, rows, op.n_aq, op.tiles, op.rp, op.col,
                                     static_cast<T *>(op.val), op.fb, op.f_idx,
                                     static_cast<T *>(op.f_v0), static_cast<T *>(op.f_v1), bin_tmp,
                                     bad);
    SCT_TRY(check_launch("k_ray_fill"));
    k_adj_fill<T><<<g, blk, 0, st>>>(n, nb, rows, op.n_aq, op.tiles, op.rp, op.col,
                                     static_cast<const T *>(op.val), bin_tmp,
                                     static_cast<T *>(op.a_v0), static_cast<T *>(op.a_v1), bad);
    SCT_TRY(check_launch("k_adj_fill"));
    SCT_TRY(grid_for(op.a_slots, 256, &g));
    SCT_TRY(grid_for(op.n_ag * op.n_aq * 4, 256, &g));
    k_adj_base<<<g, 256, 0, st>>>(bin_tmp, op.a_base, op.n_ag, op.n_aq);
    SCT_TRY(check_launch("k_adj_base"));
    SCT_TRY(grid_for(op.a_slots, 256, &g));
    k_adj_finish<<<g, 256, 0, st>>>(bin_tmp, op.a_base, op.a_rel, op.a_slots, bad);
    SCT_TRY(check_launch("k_adj_finish"));

    // Block order for the forward product.  Workgroups are dispatched to the 8
    // XCDs round-robin by block index; bundles of vertical-class rays (gathering
    // from x) go to one set of XCDs and horizontal-class ones (gathering from
    // the transposed image) to the other, in proportion to their counts.
    {
        std::vector<FwdBundle> hb(size_t(op.n_fb));
        SCT_HIP(hipMemcpyAsync(hb.data(), op.fb, sizeof(FwdBundle) * op.n_fb, hipMemcpyDeviceToHost, st));
        SCT_HIP(hipStreamSynchronize(st));
        std::vector<int32_t> V, H;
        for (int64_t b = 0; b < op.n_fb; ++b)   // empty bundles too: they write zeros
            (hb[size_t(b)].horiz ? H : V).push_back(int32_t(b));
        const int nx = 8;
        int kv = nx;
        if (!V.empty() && !H.empty()) {
            kv = int(std::lround(double(nx) * V.size() / double(V.size() + H.size())));
            kv = kv < 1 ? 1 : (kv > nx - 1 ? nx - 1 : kv);
        } else if (V.empty()) {
            kv = 0;
        }
        const int64_t rv = kv ? (int64_t(V.size()) + kv - 1) / kv : 0;
        const int64_t rh = kv < nx ? (int64_t(H.size()) + (nx - kv) - 1) / (nx - kv) : 0;
        const int64_t rounds = rv > rh ? rv : rh;
        std::vector<int32_t> order(size_t(rounds * nx > 0 ? rounds * nx : 1), -1);
        for (int64_t i = 0; i < rounds * nx; ++i) {
            const int xcd = int(i % nx);
            const int64_t j = i / nx;
            if (xcd < kv) {
                const int64_t k = j * kv + xcd;
                if (k < int64_t(V.size())) order[size_t(i)] = V[size_t(k)];
            } else {
                const int64_t k = j * (nx - kv) + (xcd - kv);
                if (k < int64_t(H.size())) order[size_t(i)] = H[size_t(k)];
            }
        }
        op.n_order = int64_t(order.size());
        SCT_TRY(op_alloc(op, reinterpret_cast<void **>(&op.fb_order), 4 * op.n_order));
        SCT_HIP(hipMemcpyAsync(op.fb_order, order.data(), 4 * order.size(), hipMemcpyHostToDevice, st));

        // Line-banded order for large images: (bundle, band) items, band-major
        // within each gather class, on the same XCD split.  Item (B, band)
        // exists when a quad of B starts in the band.
        if (op.n >= kBandMinN) {
            op.n_bands = (op.n + kBandLines - 1) / kBandLines;
            std::vector<int2> BV, BH;
            for (int band = 0; band < op.n_bands; ++band)
                for (int64_t b = 0; b < op.n_fb; ++b) {
                    const FwdBundle &d = hb[size_t(b)];
                    if (d.nrows <= 0) continue;
                    const int lo = d.m0 / kBandLines, hi = (d.m0 + d.nrows - 4) / kBandLines;
                    if (band < lo || band > hi) continue;
                    (d.horiz ? BH : BV).push_back(make_int2(int(b), band));
                }
            const int64_t bv = kv ? (int64_t(BV.size()) + kv - 1) / kv : 0;
            const int64_t bh = kv < nx ? (int64_t(BH.size()) + (nx - kv) - 1) / (nx - kv) : 0;
            const int64_t brounds = bv > bh ? bv : bh;
            std::vector<int2> border(size_t(brounds * nx > 0 ? brounds * nx : 1), make_int2(-1, -1));
            for (int64_t i = 0; i < brounds * nx; ++i) {
                const int xcd = int(i % nx);
                const int64_t j = i / nx;
                if (xcd < kv) {
                    const int64_t k = j * kv + xcd;
                    if (k < int64_t(BV.size())) border[size_t(i)] = BV[size_t(k)];
                } else {
                    const int64_t k = j * (nx - kv) + (xcd - kv);
                    if (k < int64_t(BH.size())) border[size_t(i)] = BH[size_t(k)];
                }
            }
            op.n_band_order = int64_t(border.size());
            SCT_TRY(op_alloc(op, reinterpret_cast<void **>(&op.fb_band_order), 8 * op.n_band_order));
            SCT_HIP(hipMemcpyAsync(op.fb_band_order, border.data(), 8 * border.size(),
                                   hipMemcpyHostToDevice, st));
        }
    }

    int32_t bad_h = 0;
    SCT_HIP(hipMemcpyAsync(&bad_h, bad, 4, hipMemcpyDeviceToHost, st));
    SCT_HIP(hipStreamSynchronize(st));
    if (bad_h)
        return set_error(RADON_EUNSUPPORTED,
                         "slotted layout assumption violated (code %d): a ray met more than two "
                         "pixels of one line, or a pixel more than two bins of one angle", bad_h);
    return RADON_OK;
}

}  // namespace sct

using namespace sct;

extern "C" const char *radon_last_error(void) { return sct::last_error(); }

extern "C" int build_radon_csr(const radon_geom *g, void *stream, radon_op **out)
{
    clear_error();
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return set_error(RADON_EINVAL, "geometry is NULL");
    if (g->n < 1 || g->n > 32767) return set_error(RADON_EINVAL, "n must be in [1, 32767] (got %d)", g->n);
    if (g->n_angles < 1) return set_error(RADON_EINVAL, "n_angles must be >= 1 (got %d)", g->n_angles);
    if (g->n_bins < 1 || g->n_bins > 65535)
        return set_error(RADON_EINVAL, "n_bins must be in [1, 65535] (got %d)", g->n_bins);
    if (g->dtype != SPARSECT_F32 && g->dtype != SPARSECT_F64 && g->dtype != SPARSECT_F32_F64)
        return set_error(RADON_EINVAL, "dtype must be SPARSECT_F32, SPARSECT_F64 or SPARSECT_F32_F64 (got %d)",
                         g->dtype);
    std::vector<int32_t> meas;
    for (int k = 0; k < g->n_angles; ++k)
        if (!g->measured || g->measured[k]) meas.push_back(k);
    if (meas.empty()) return set_error(RADON_EINVAL, "no measured angle");
    const int64_t rows = int64_t(meas.size()) * g->n_bins;
    if (rows >= INT_MAX) return set_error(RADON_EOVERFLOW, "measured rays %lld exceed int32", (long long)rows);
    const int64_t nn = int64_t(g->n) * g->n;
    const int64_t aslots = int64_t((g->n + 7) / 8) * ((g->n + 7) / 8) * 64 * 4 *
                           ((int64_t(meas.size()) + 3) / 4);
    if (aslots >= (int64_t(1) << 40)) return set_error(RADON_EOVERFLOW, "adjoint layout too large");

    Op *op = new (std::nothrow) Op();
    if (!op) return set_error(RADON_EINVAL, "out of host memory");
    op->n = g->n;
    op->n_angles = g->n_angles;
    op->n_bins = g->n_bins;
    op->dtype = g->dtype;
    op->meas = meas;
    op->n_meas = int32_t(meas.size());
    op->nn = nn;
    op->rows = rows;
    op->msize = g->dtype == SPARSECT_F64 ? 8 : 4;
    op->vsize = g->dtype == SPARSECT_F32 ? 4 : 8;

    std::vector<double> cs(2 * meas.size());
    for (size_t a = 0; a < meas.size(); ++a) {
        angle_cos_sin(meas[a], g->n_angles, &cs[2 * a], &cs[2 * a + 1]);
        if (std::fabs(cs[2 * a + 1]) > std::fabs(cs[2 * a])) op->need_T = true;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc;
    try {
        rc = op->msize == 4 ? build_typed<float>(*op, cs, st) : build_typed<double>(*op, cs, st);
    } catch (...) {
        rc = set_error(RADON_EINVAL, "unexpected host exception during build");
    }
    if (rc != RADON_OK) {
        (void)hipStreamSynchronize(st);
        op_free(op);
        return rc;
    }
    *out = reinterpret_cast<radon_op *>(op);
    return RADON_OK;
}

extern "C" void radon_op_destroy(radon_op *p) { op_free(as_op(p)); }

extern "C" int radon_op_info(const radon_op *p, radon_info *out)
{
    clear_error();
    SCT_TRY(check_op(p));
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    const Op *op = as_op(p);
    out->n_pixels = op->nn;
    out->n_meas_angles = op->n_meas;
    out->n_meas_rays = op->rows;
    out->nnz = op->nnz;
    out->fwd_slots = op->f_slots;
    out->adj_slots = op->a_slots;
    out->device_bytes = op->device_bytes;
    out->dtype = op->dtype;
    out->n = op->n;
    out->n_angles = op->n_angles;
    out->n_bins = op->n_bins;
    out->needs_transpose = op->need_T ? 1 : 0;
    out->reserved = 0;
    return RADON_OK;
}

template <class T>
static int export_csr_typed(const Op &op, int64_t *rp, int32_t *col, double *val)
{
    if (rp) SCT_HIP(hipMemcpy(rp, op.rp, size_t(8 * (op.rows + 1)), hipMemcpyDeviceToHost));
    if (col) SCT_HIP(hipMemcpy(col, op.col, size_t(4 * op.nnz), hipMemcpyDeviceToHost));
    if (val) {
        std::vector<T> v(size_t(op.nnz));
        SCT_HIP(hipMemcpy(v.data(), op.val, size_t(sizeof(T) * op.nnz), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < op.nnz; ++i) val[i] = double(v[size_t(i)]);
    }
    return RADON_OK;
}

extern "C" int radon_export_csr(const radon_op *p, int64_t *row_ptr, int32_t *col, double *val)
{
    clear_error();
    SCT_TRY(check_op(p));
    const Op &op = *as_op(p);
    try {
        return op.msize == 4 ? export_csr_typed<float>(op, row_ptr, col, val)
                             : export_csr_typed<double>(op, row_ptr, col, val);
    } catch (...) {
        return set_error(RADON_EINVAL, "out of host memory");
    }
}

template <class T>
static int export_adj_typed(const Op &op, int32_t *bin, double *v0, double *v1)
{
    const size_t ns = size_t(op.a_slots);
    std::vector<uint8_t> rel(ns);
    std::vector<uint16_t> base(size_t(op.n_ag * op.n_aq * 4));
    std::vector<T> a0(ns), a1(ns);
    SCT_HIP(hipMemcpy(rel.data(), op.a_rel, ns, hipMemcpyDeviceToHost));
    SCT_HIP(hipMemcpy(base.data(), op.a_base, 2 * base.size(), hipMemcpyDeviceToHost));
    SCT_HIP(hipMemcpy(a0.data(), op.a_v0, sizeof(T) * ns, hipMemcpyDeviceToHost));
    SCT_HIP(hipMemcpy(a1.data(), op.a_v1, sizeof(T) * ns, hipMemcpyDeviceToHost));
    for (int64_t j = 0; j < op.nn; ++j)
        for (int a = 0; a < op.n_meas; ++a) {
            const size_t s = size_t(adj_slot(int(j / op.n), int(j % op.n), a, op.n_aq, op.tiles));
            const size_t bi = ((s >> 2) / kAdjLanes) * 4 + (s & 3);
            const size_t o = size_t(j * op.n_meas + a);
            const bool empty = a0[s] == T(0) && a1[s] == T(0);
            if (bin) bin[o] = empty ? -1 : int32_t(base[bi]) + int32_t(rel[s]);
            if (v0) v0[o] = double(a0[s]);
            if (v1) v1[o] = double(a1[s]);
        }
    return RADON_OK;
}

extern "C" int radon_export_adj(const radon_op *p, int32_t *bin, double *v0, double *v1)
{
    clear_error();
    SCT_TRY(check_op(p));
    const Op &op = *as_op(p);
    try {
        return op.msize == 4 ? export_adj_typed<float>(op, bin, v0, v1)
                             : export_adj_typed<double>(op, bin, v0, v1);
    } catch (...) {
        return set_error(RADON_EINVAL, "out of host memory");
    }
}
