// Operator construction: Siddon ray tracing on the GPU, the CSR of MR, and the
// two slotted layouts the apply kernels stream (Section 3 of the paper: the
// sparse operator is precomputed once for a fixed geometry).
//
// This file is compiled with FP contraction off so that every crossing
// parameter and length is computed with the plain IEEE operations of its
// formula.
#include "internal.hpp"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>

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

// Pass 1: entries per measured ray, the range of major lines it covers and
// its chord: the summed length on its second line when a third follows (that
// line is crossed from side to side), else 0.
__global__ void k_ray_count(const double2 *__restrict__ cs, int n, int nb, int64_t rows,
                            int64_t *__restrict__ cnt, int32_t *__restrict__ mlo,
                            int32_t *__restrict__ mhi, double *__restrict__ chord)
{
    const int64_t ray = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ray >= rows) return;
    const int a = int(ray / nb), b = int(ray % nb);
    const double c = cs[a].x, s = cs[a].y;
    const double sb = double(b) - 0.5 * double(nb - 1);
    const bool hz = is_horiz(c, s);
    int64_t count = 0;
    int lo = INT_MAX, hi = -1;
    int cur = -1, lines = 0;
    double lsum = 0.0, ch = 0.0;
    trace_ray(n, c, s, sb, [&](int j, double len) {
        ++count;
        const int m = hz ? j % n : j / n;
        lo = m < lo ? m : lo;
        hi = m > hi ? m : hi;
        if (m != cur) {
            if (lines == 2) ch = lsum;   // the second line is complete and not the last
            ++lines;
            cur = m;
            lsum = len;
        } else {
            lsum += len;
        }
    });
    cnt[ray] = count;
    mlo[ray] = lo;
    mhi[ray] = hi;
    chord[ray] = ch;
}

// Bundle extents: union of the major ranges of the bundle's rays (up to R
// adjacent bins of each of its angles).
__global__ void k_bundle_span(const double2 *__restrict__ cs, const int32_t *__restrict__ mlo,
                              const int32_t *__restrict__ mhi, int nb, BundleMap bm, int bw, int64_t n_fb,
                              FwdBundle *__restrict__ fb, int64_t *__restrict__ slots)
{
    const int64_t B = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (B >= n_fb) return;
    int a0 = 0, na = 0;
    bm.group(B / bm.nbpr, &a0, &na);
    const int t = int(B % bm.nbpr);
    const int ray0 = a0 * nb + t * bm.rpa;
    const int nrays = min(bm.rpa, nb - t * bm.rpa);
    int lo = INT_MAX, hi = -1;
    for (int j = 0; j < na; ++j) {
        for (int r = 0; r < nrays; ++r) {
            const int ray = ray0 + j * nb + r;
            if (mhi[ray] >= 0) {
                lo = min(lo, mlo[ray]);
                hi = max(hi, mhi[ray]);
            }
        }
    }
    FwdBundle d;
    d.off = 0;
    d.m0 = hi >= 0 ? lo : 0;
    d.nrows = hi >= 0 ? ((hi - lo + 1 + 3) / 4) * 4 : 0;
    d.ray0 = ray0;
    d.astride = nb;
    d.nrays = int16_t(nrays);
    d.nang = int16_t(na);
    d.rshift = int16_t(__builtin_ctz(unsigned(bm.rpa)));
    d.horiz = is_horiz(cs[a0].x, cs[a0].y) ? 1 : 0;
    fb[B] = d;
    slots[B] = int64_t(d.nrows) * bw;
}

__global__ void k_bundle_off(FwdBundle *__restrict__ fb, const int64_t *__restrict__ incl,
                             int64_t n_fb, int bw)
{
    const int64_t B = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (B >= n_fb) return;
    fb[B].off = incl[B] - int64_t(fb[B].nrows) * bw;
}

// Relative tolerance of the chord check: lengths on one line add up to the
// chord to within the rounding of the FP64 ray parameters (about 1e-13 of the
// image side) and the dropped slivers (below kSliver).
constexpr double kChordTol = 1e-9;

// Pass 2: write the CSR row, the ray's forward slots (first pixel, its
// length and, unless the operator is compact (f_v1 == nullptr), the second
// length) and its RayEdge, and mark the first bin of every (pixel, angle)
// pair the ray touches.  Every line between the ray's first and last must
// hold the chord (bad flag 32 otherwise: a compact forward derives the
// second length from it).
template <class T>
__global__ void k_ray_fill(const double2 *__restrict__ cs, int n, int nb, BundleMap bm, int bw, int64_t rows,
                           int n_aq, int tiles, const int64_t *__restrict__ rp, int32_t *__restrict__ col,
                           T *__restrict__ val, const FwdBundle *__restrict__ fb,
                           uint16_t *__restrict__ f_idx, T *__restrict__ f_v0, T *__restrict__ f_v1,
                           const int32_t *__restrict__ mlo, const int32_t *__restrict__ mhi,
                           const double *__restrict__ chord, RayEdge *__restrict__ f_edge,
                           int n_stored, int n_adj_ang, int32_t *__restrict__ bin_tmp,
                           int32_t *__restrict__ bad)
{
    const int64_t ray = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ray >= rows) return;
    const int a = int(ray / nb), b = int(ray % nb);
    const double c = cs[a].x, s = cs[a].y;
    const double sb = double(b) - 0.5 * double(nb - 1);
    const bool hz = is_horiz(c, s);
    // rays of angles without bundles of their own (a symmetric operator's
    // partners) get no slots
    const bool slotted = a < n_stored;
    int r = 0;
    FwdBundle d{};
    if (slotted) d = fb[bm.bundle_of(a, b, &r)];
    const int mf = mlo[ray], ml = mhi[ray];
    const double ch = chord[ray];
    RayEdge e;
    e.chord = ch;
    e.w1f = 0.0;
    e.w1l = 0.0;
    e.mf = ml >= 0 ? mf : 1;   // no pixels: mf > ml
    e.ml = ml >= 0 ? ml : 0;
    int64_t o = rp[ray];
    int cur = -1, nline = 0, q0 = 0, q1 = 0;
    T w0 = T(0), w1 = T(0);
    double l0 = 0.0, l1 = 0.0;
    const int64_t oend = rp[ray + 1];
    auto flush = [&]() {
        if (cur < 0) return;
        if (slotted && (cur < d.m0 || cur >= d.m0 + d.nrows)) {
            atomicOr(bad, 16);
            return;
        }
        T v1 = T(0);
        int first = q0;
        T v0 = w0;
        if (nline != 1) {
            if (q1 != q0 + 1 && q0 != q1 + 1) atomicOr(bad, 1);
            const bool first0 = q0 < q1;
            first = first0 ? q0 : q1;
            v0 = first0 ? w0 : w1;
            v1 = first0 ? w1 : w0;
        }
        if (slotted) {
            const int64_t slot = fwd_slot(d.off, cur - d.m0, r, bw);
            f_idx[slot] = uint16_t(first);
            f_v0[slot] = v0;
            if (f_v1) f_v1[slot] = v1;
        }
        if (cur == mf) e.w1f = double(v1);
        if (cur == ml) e.w1l = double(v1);
        if (cur != mf && cur != ml && !(fabs(l0 + l1 - ch) <= kChordTol * ch)) atomicOr(bad, 32);
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
            l0 = len;
            l1 = 0.0;
        } else {
            if (nline >= 2) atomicOr(bad, 2);
            nline = 2;
            q1 = q;
            w1 = v;
            l1 = len;
        }
        if (a < n_adj_ang) atomicMin(&bin_tmp[adj_slot(j / n, j % n, a, n_aq, tiles)], b);
    });
    flush();
    if (o != oend) atomicOr(bad, 4);
    f_edge[ray] = e;
}

// Pass 3: place each entry in its (pixel, angle) slot as the first or second bin.
template <class T>
__global__ void k_adj_fill(int n, int nb, int64_t rows, int n_aq, int tiles, int n_adj_ang,
                           const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const T *__restrict__ val, const int32_t *__restrict__ bin_tmp, T *__restrict__ a_v0,
                           T *__restrict__ a_v1, int32_t *__restrict__ bad)
{
    const int64_t ray = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ray >= rows) return;
    const int a = int(ray / nb), b = int(ray % nb);
    if (a >= n_adj_ang) return;   // a partner angle of an adjoint stored by symmetry
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

// Device memory of a build.  Every array comes either from buffers the caller
// allocated (build_radon_csr_into: the CSR arrays, one block for the derived
// layouts and one workspace) or from allocations the handle owns
// (build_radon_csr); temporaries always come from the workspace.
struct Carve {
    char *base = nullptr;
    int64_t cap = 0, used = 0;
    const char *what = "";
    template <class T>
    int take(T **p, int64_t bytes)
    {
        used = (used + 255) & ~int64_t(255);
        if (bytes <= 0) bytes = 1;
        if (used + bytes > cap)
            return set_error(RADON_EWORKSPACE, "%s: %lld bytes are not enough", what, (long long)cap);
        *p = reinterpret_cast<T *>(base + used);
        used += bytes;
        return RADON_OK;
    }
};

// Sizes known once the rays are counted, and the host-side work orders.
struct Plan {
    int64_t nnz = 0, fslots = 0;
    std::vector<int32_t> order;   // block -> bundle of the forward product
    std::vector<int2> border[4];  // (bundle, band) items of the line-banded forward, per height
    std::vector<int32_t> aorder;  // adjoint tile order of the fused products
    std::vector<AdjOrbit> orbs;   // tile orbits of an adjoint stored by symmetry
};

static int64_t up256(int64_t b) { return (b + 255) & ~int64_t(255); }

// Bytes of hipcub's scan temporaries for the two scans of the count phase.
static int scan_bytes(int64_t rows, int64_t n_fb, size_t *out)
{
    size_t a = 0, b = 0;
    int64_t *dummy = nullptr;
    SCT_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, a, dummy, dummy, rows, hipStream_t(nullptr)));
    SCT_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, b, dummy, dummy, n_fb, hipStream_t(nullptr)));
    *out = a > b ? a : b;
    return RADON_OK;
}

static int64_t n_fb_of(const Op &op) { return op.bmap.bundles(); }

// Workspace of a build: room for the row pointers and the bundle table (the
// sizes query keeps them there), the count-phase arrays and the temporary
// first-bin table of the adjoint layout.
static int build_ws_bytes(const Op &op, int64_t *out)
{
    const int64_t rows = op.rows, n_fb = n_fb_of(op);
    size_t sb = 0;
    SCT_TRY(scan_bytes(rows, n_fb, &sb));
    int64_t b = 0;
    b += up256(8 * (rows + 1));                           // row pointers (sizes query)
    b += up256(int64_t(sizeof(FwdBundle)) * n_fb);        // bundle table (sizes query)
    b += up256(16 * int64_t(op.n_meas));                  // (cos, sin)
    b += up256(8 * rows) + 2 * up256(4 * rows);           // counts, major-line ranges
    b += up256(8 * rows);                                 // chords
    b += up256(4);                                        // error flags
    b += 2 * up256(8 * n_fb);                             // bundle slots and their scan
    b += up256(int64_t(sb));                              // scan temporaries
    b += up256(4 * op.a_slots);                           // first-bin table
    *out = b;
    return RADON_OK;
}

// Bytes of the derived layouts for a plan.
static int64_t layout_bytes(const Op &op, const Plan &pl)
{
    const int64_t es = op.msize;
    int64_t b = 0;
    b += up256(int64_t(sizeof(FwdBundle)) * n_fb_of(op));
    b += up256(2 * pl.fslots) + (op.compact ? 1 : 2) * up256(es * pl.fslots);
    b += up256(int64_t(sizeof(RayEdge)) * op.rows);
    if (op.sym) b += up256(16 * int64_t(op.n_rep));
    b += up256(op.a_slots) + up256(2 * op.n_ag * op.n_aq * 4) + 2 * up256(es * op.a_slots);
    b += up256(4 * int64_t(pl.order.size()));
    for (const auto &bo : pl.border) b += up256(8 * int64_t(bo.size()));
    b += up256(4 * int64_t(pl.aorder.size()));
    b += up256(int64_t(sizeof(AdjOrbit)) * int64_t(pl.orbs.size()));
    return b;
}

// Temporaries of the count phase, carved from the workspace after the slots
// for the row pointers and the bundle table.
struct CountTmp {
    double2 *cs = nullptr;
    int64_t *cnt = nullptr, *bslots = nullptr, *bincl = nullptr;
    int32_t *mlo = nullptr, *mhi = nullptr, *bad = nullptr;
    double *chord = nullptr;
    void *scan = nullptr;
    size_t scan_bytes = 0;
    int32_t *bin_tmp = nullptr;
};

// Count phase: entries per ray into rp (scanned into row pointers), the bundle
// table fb with each bundle's slot offset, then (host) nnz, the forward slot
// count and the work orders.  Synchronises the stream.
static int count_phase(Op &op, const std::vector<double> &cs_host, hipStream_t st, Carve &ws,
                       int64_t *rp, FwdBundle *fb, CountTmp &t, Plan &pl)
{
    const int n = op.n, nb = op.n_bins;
    const int64_t rows = op.rows;
    const int blk = 128;
    unsigned g;
    op.n_fb = n_fb_of(op);

    SCT_TRY(ws.take(&t.cs, int64_t(sizeof(double2)) * op.n_meas));
    SCT_TRY(ws.take(&t.cnt, 8 * rows));
    SCT_TRY(ws.take(&t.mlo, 4 * rows));
    SCT_TRY(ws.take(&t.mhi, 4 * rows));
    SCT_TRY(ws.take(&t.chord, 8 * rows));
    SCT_TRY(ws.take(&t.bad, 4));
    SCT_TRY(ws.take(&t.bslots, 8 * op.n_fb));
    SCT_TRY(ws.take(&t.bincl, 8 * op.n_fb));
    SCT_TRY(scan_bytes(rows, op.n_fb, &t.scan_bytes));
    SCT_TRY(ws.take(&t.scan, int64_t(t.scan_bytes)));
    SCT_TRY(ws.take(&t.bin_tmp, 4 * op.a_slots));

    SCT_HIP(hipMemcpyAsync(t.cs, cs_host.data(), sizeof(double2) * op.n_meas, hipMemcpyHostToDevice, st));
    SCT_HIP(hipMemsetAsync(t.bad, 0, 4, st));
    SCT_TRY(grid_for(rows, blk, &g));
    k_ray_count<<<g, blk, 0, st>>>(t.cs, n, nb, rows, t.cnt, t.mlo, t.mhi, t.chord);
    SCT_TRY(check_launch("k_ray_count"));

    SCT_HIP(hipMemsetAsync(rp, 0, 8, st));
    size_t sb = t.scan_bytes;
    SCT_HIP(hipcub::DeviceScan::InclusiveSum(t.scan, sb, t.cnt, rp + 1, rows, st));
    SCT_TRY(grid_for(op.n_fb, blk, &g));
    k_bundle_span<<<g, blk, 0, st>>>(t.cs, t.mlo, t.mhi, nb, op.bmap, op.bw, op.n_fb, fb, t.bslots);
    SCT_TRY(check_launch("k_bundle_span"));
    sb = t.scan_bytes;
    SCT_HIP(hipcub::DeviceScan::InclusiveSum(t.scan, sb, t.bslots, t.bincl, op.n_fb, st));
    k_bundle_off<<<g, blk, 0, st>>>(fb, t.bincl, op.n_fb, op.bw);
    SCT_TRY(check_launch("k_bundle_off"));

    SCT_HIP(hipMemcpyAsync(&pl.nnz, rp + rows, 8, hipMemcpyDeviceToHost, st));
    SCT_HIP(hipMemcpyAsync(&pl.fslots, t.bincl + (op.n_fb - 1), 8, hipMemcpyDeviceToHost, st));
    std::vector<FwdBundle> hb(size_t(op.n_fb));
    SCT_HIP(hipMemcpyAsync(hb.data(), fb, sizeof(FwdBundle) * op.n_fb, hipMemcpyDeviceToHost, st));
    SCT_HIP(hipStreamSynchronize(st));
    if (pl.nnz >= (int64_t(1) << 40)) return set_error(RADON_EOVERFLOW, "nnz %lld too large", (long long)pl.nnz);

    // Block order for the forward product.  Workgroups are dispatched to the 8
    // XCDs round-robin by block index; bundles of vertical-class rays (gathering
    // from x) go to one set of XCDs and horizontal-class ones (gathering from
    // the transposed image) to the other, in proportion to their counts.
    // Within each class the bundles go longest first: block i takes entries
    // i, i + G, ... of the list, so every block gets one of the longest
    // bundles of its class, then one of the next longest, and so on, and no
    // block is left at the end with several long bundles while the others
    // idle (in bundle order the busiest of the 2048 blocks of the
    // 512 x 512 / 180-angle operator had about 1.45x the mean work, longest
    // first 1.19x; the forward went from 96.9 to 93.8 us at 16 rays per
    // bundle and to 89.5 us at 64).
    std::vector<int32_t> V, H;
    for (int64_t b = 0; b < op.n_fb; ++b)   // empty bundles too: they write zeros
        (hb[size_t(b)].horiz ? H : V).push_back(int32_t(b));
    const auto longer = [&](int32_t a, int32_t c) { return hb[size_t(a)].nrows > hb[size_t(c)].nrows; };
    std::stable_sort(V.begin(), V.end(), longer);
    std::stable_sort(H.begin(), H.end(), longer);
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
    pl.order.assign(size_t(rounds * nx > 0 ? rounds * nx : 1), -1);
    for (int64_t i = 0; i < rounds * nx; ++i) {
        const int xcd = int(i % nx);
        const int64_t j = i / nx;
        if (xcd < kv) {
            const int64_t k = j * kv + xcd;
            if (k < int64_t(V.size())) pl.order[size_t(i)] = V[size_t(k)];
        } else {
            const int64_t k = j * (nx - kv) + (xcd - kv);
            if (k < int64_t(H.size())) pl.order[size_t(i)] = H[size_t(k)];
        }
    }

    // Line-banded orders: (bundle, band) items, band-major within each gather
    // class, on the same XCD split, one list per band height.  Item (B, band)
    // exists when a quad of B starts in the band.
    for (int h = 0; h < 4; ++h) {
        pl.border[h].clear();
        if (op.n < kBandSetMinN) continue;
        const int L = kBandHeights[h];
        const int n_bands = (op.n + L - 1) / L;
        std::vector<int2> BV, BH;
        for (int band = 0; band < n_bands; ++band)
            for (int64_t b = 0; b < op.n_fb; ++b) {
                const FwdBundle &d = hb[size_t(b)];
                if (d.nrows <= 0) continue;
                const int lo = d.m0 / L, hi = (d.m0 + d.nrows - 4) / L;
                if (band < lo || band > hi) continue;
                (d.horiz ? BH : BV).push_back(make_int2(int(b), band));
            }
        const int64_t bv = kv ? (int64_t(BV.size()) + kv - 1) / kv : 0;
        const int64_t bh = kv < nx ? (int64_t(BH.size()) + (nx - kv) - 1) / (nx - kv) : 0;
        const int64_t brounds = bv > bh ? bv : bh;
        std::vector<int2> &border = pl.border[h];
        border.assign(size_t(brounds * nx > 0 ? brounds * nx : 1), make_int2(-1, -1));
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
    }

    // Adjoint tile order of the fused products: tiles by Morton code of
    // (tile row, tile column), cut into 8 consecutive runs; entry i belongs to
    // run i % 8, so the workgroups of XCD x walk run x.
    {
        const int T = op.tiles;
        std::vector<std::pair<uint64_t, int32_t>> mt;
        mt.reserve(size_t(op.n_ag));
        for (int ty = 0; ty < T; ++ty)
            for (int tx = 0; tx < T; ++tx) {
                uint64_t code = 0;
                for (int bit = 0; bit < 16; ++bit)
                    code |= (uint64_t((tx >> bit) & 1) << (2 * bit)) | (uint64_t((ty >> bit) & 1) << (2 * bit + 1));
                mt.emplace_back(code, ty * T + tx);
            }
        std::sort(mt.begin(), mt.end());
        if (op.sym_adj) {
            // An adjoint stored by symmetry: tile g reads the slots of its
            // images under x -> -x, the transpose and both, so the tiles of
            // one orbit under those maps (8, or 4 or 1 on the diagonals and
            // the middle lines) read the same slots.  Orbits fill groups of 8
            // entries (whole orbits of 8 first, in the Morton order of their
            // first tile, then the smaller ones by decreasing size, which
            // packs them without gaps); group i goes to XCD i % 8 with its
            // entries at r*64 + i%8 + 8k (r = i / 8): the workgroups of one
            // XCD take an orbit's tiles at once, so all but the first reader
            // of a slot find it in L2.
            std::vector<char> seen(size_t(op.n_ag), 0);
            std::vector<std::vector<int32_t>> small;
            pl.orbs.clear();
            std::vector<int32_t> flat;   // orbit tiles, groups of 8 (-1: unused)
            for (const auto &m : mt) {
                if (seen[size_t(m.second)]) continue;
                std::vector<int32_t> orb(1, m.second);
                seen[size_t(m.second)] = 1;
                for (size_t h = 0; h < orb.size(); ++h) {
                    const int tx = orb[h] % T, ty = orb[h] / T;
                    const int32_t img[2] = {ty * T + (T - 1 - tx), tx * T + ty};
                    for (int32_t u : img)
                        if (!seen[size_t(u)]) {
                            seen[size_t(u)] = 1;
                            orb.push_back(u);
                        }
                }
                // the orbit table: for output tile t and each map, the
                // source tile k_adj1_sym reads (for k_adj1_orb)
                AdjOrbit ob;
                for (int k = 0; k < 8; ++k) ob.tile[k] = k < int(orb.size()) ? orb[size_t(k)] : -1;
                for (size_t ti = 0; ti < 8; ++ti)
                    for (int m = 0; m < 4; ++m) ob.src[ti][m] = 0;
                for (size_t ti = 0; ti < orb.size(); ++ti) {
                    const int tx = orb[ti] % T, ty = orb[ti] / T;
                    const int32_t src[4] = {orb[ti], ty * T + (T - 1 - tx), tx * T + ty, (T - 1 - tx) * T + ty};
                    for (int m = 0; m < 4; ++m) {
                        size_t at = 0;
                        while (orb[at] != src[m]) ++at;   // the orbit is closed under the maps
                        ob.src[ti][m] = uint8_t(at);
                    }
                }
                pl.orbs.push_back(ob);
                if (orb.size() == 8) flat.insert(flat.end(), orb.begin(), orb.end());
                else small.push_back(std::move(orb));
            }
            std::stable_sort(small.begin(), small.end(),
                             [](const std::vector<int32_t> &a, const std::vector<int32_t> &b) {
                                 return a.size() > b.size();
                             });
            for (const auto &orb : small) flat.insert(flat.end(), orb.begin(), orb.end());
            flat.resize((flat.size() + 7) / 8 * 8, -1);
            const int64_t groups = int64_t(flat.size()) / 8;
            pl.aorder.assign(size_t((groups + nx - 1) / nx * 64), -1);
            for (int64_t i = 0; i < groups; ++i)
                for (int k = 0; k < 8; ++k)
                    pl.aorder[size_t((i / nx) * 64 + i % nx + 8 * k)] = flat[size_t(i * 8 + k)];
        } else {
            const int64_t per = (op.n_ag + nx - 1) / nx;
            pl.aorder.assign(size_t(per * nx), -1);
            for (int64_t r = 0; r < nx; ++r)
                for (int64_t j = 0; j < per; ++j) {
                    const int64_t k = r * per + j;
                    if (k < op.n_ag) pl.aorder[size_t(j * nx + r)] = mt[size_t(k)].second;
                }
        }
    }
    return RADON_OK;
}

// Fill phase: the CSR entries, both slotted layouts and the work orders, into
// the arrays already set on op (rp, col, val, fb and the layout arrays).
// Synchronises the stream.
template <class T>
static int fill_phase(Op &op, const Plan &pl, hipStream_t st, const CountTmp &t)
{
    const int n = op.n, nb = op.n_bins;
    const int64_t rows = op.rows;
    const int blk = 128;
    const int64_t es = sizeof(T);
    unsigned g;
    SCT_HIP(hipMemsetAsync(op.f_idx, 0, size_t(2 * op.f_slots), st));
    SCT_HIP(hipMemsetAsync(op.f_v0, 0, size_t(es * op.f_slots), st));
    if (op.f_v1) SCT_HIP(hipMemsetAsync(op.f_v1, 0, size_t(es * op.f_slots), st));
    SCT_HIP(hipMemsetAsync(op.a_v0, 0, size_t(es * op.a_slots), st));
    SCT_HIP(hipMemsetAsync(op.a_v1, 0, size_t(es * op.a_slots), st));
    SCT_HIP(hipMemsetAsync(t.bin_tmp, 0x7f, size_t(4 * op.a_slots), st));   // 0x7f7f7f7f > any bin

    SCT_TRY(grid_for(rows, blk, &g));
    k_ray_fill<T><<<g, blk, 0, st>>>(t.cs, n, nb, op.bmap, op.bw, rows, op.n_aq, op.tiles, op.rp, op.col,
                                     static_cast<T *>(op.val), op.fb, op.f_idx,
                                     static_cast<T *>(op.f_v0), static_cast<T *>(op.f_v1), t.mlo, t.mhi,
                                     t.chord, op.f_edge, op.sym ? op.n_rep : op.n_meas, op.n_adj_ang,
                                     t.bin_tmp, t.bad);
    SCT_TRY(check_launch("k_ray_fill"));
    k_adj_fill<T><<<g, blk, 0, st>>>(n, nb, rows, op.n_aq, op.tiles, op.n_adj_ang, op.rp, op.col,
                                     static_cast<const T *>(op.val), t.bin_tmp,
                                     static_cast<T *>(op.a_v0), static_cast<T *>(op.a_v1), t.bad);
    SCT_TRY(check_launch("k_adj_fill"));
    SCT_TRY(grid_for(op.n_ag * op.n_aq * 4, 256, &g));
    k_adj_base<<<g, 256, 0, st>>>(t.bin_tmp, op.a_base, op.n_ag, op.n_aq);
    SCT_TRY(check_launch("k_adj_base"));
    SCT_TRY(grid_for(op.a_slots, 256, &g));
    k_adj_finish<<<g, 256, 0, st>>>(t.bin_tmp, op.a_base, op.a_rel, op.a_slots, t.bad);
    SCT_TRY(check_launch("k_adj_finish"));

    SCT_HIP(hipMemcpyAsync(op.fb_order, pl.order.data(), 4 * pl.order.size(), hipMemcpyHostToDevice, st));
    if (op.sym)
        SCT_HIP(hipMemcpyAsync(op.f_partner, op.partner_host.data(), 16 * op.partner_host.size(),
                               hipMemcpyHostToDevice, st));
    for (int h = 0; h < 4; ++h)
        if (op.bands[h].n_bands > 0)
            SCT_HIP(hipMemcpyAsync(op.bands[h].order, pl.border[h].data(), 8 * pl.border[h].size(),
                                   hipMemcpyHostToDevice, st));
    SCT_HIP(hipMemcpyAsync(op.a_order, pl.aorder.data(), 4 * pl.aorder.size(), hipMemcpyHostToDevice, st));
    if (op.n_orb)
        SCT_HIP(hipMemcpyAsync(op.a_orb, pl.orbs.data(), sizeof(AdjOrbit) * pl.orbs.size(), hipMemcpyHostToDevice,
                               st));

    int32_t bad_h = 0;
    SCT_HIP(hipMemcpyAsync(&bad_h, t.bad, 4, hipMemcpyDeviceToHost, st));
    SCT_HIP(hipStreamSynchronize(st));
    if (bad_h)
        return set_error(RADON_EUNSUPPORTED,
                         "slotted layout assumption violated (code %d): a ray met more than two "
                         "pixels of one line, a pixel more than two bins of one angle, or a line "
                         "inside a ray's range held other than the ray's chord (32)", bad_h);
    return RADON_OK;
}

// Point op's derived-layout arrays into `lay` (which already holds the bundle
// table at its start when `fb_taken`), after the plan is known.
static int carve_layouts(Op &op, const Plan &pl, Carve &lay, bool fb_taken)
{
    const int64_t es = op.msize;
    if (!fb_taken) SCT_TRY(lay.take(&op.fb, int64_t(sizeof(FwdBundle)) * op.n_fb));
    SCT_TRY(lay.take(&op.f_idx, 2 * pl.fslots));
    SCT_TRY(lay.take(&op.f_v0, es * pl.fslots));
    op.f_v1 = nullptr;
    if (!op.compact) SCT_TRY(lay.take(&op.f_v1, es * pl.fslots));
    SCT_TRY(lay.take(&op.f_edge, int64_t(sizeof(RayEdge)) * op.rows));
    op.f_partner = nullptr;
    if (op.sym) SCT_TRY(lay.take(&op.f_partner, 16 * int64_t(op.n_rep)));
    SCT_TRY(lay.take(&op.a_rel, op.a_slots));
    SCT_TRY(lay.take(&op.a_base, 2 * op.n_ag * op.n_aq * 4));
    SCT_TRY(lay.take(&op.a_v0, es * op.a_slots));
    SCT_TRY(lay.take(&op.a_v1, es * op.a_slots));
    op.n_order = int64_t(pl.order.size());
    SCT_TRY(lay.take(&op.fb_order, 4 * op.n_order));
    for (int h = 0; h < 4; ++h) {
        BandSet &b = op.bands[h];
        b.lines = kBandHeights[h];
        b.n_bands = pl.border[h].empty() ? 0 : (op.n + b.lines - 1) / b.lines;
        b.n_order = int64_t(pl.border[h].size());
        b.order = nullptr;
        if (b.n_bands > 0) SCT_TRY(lay.take(&b.order, 8 * b.n_order));
    }
    static_assert(kBandHeights[0] == kBandLines, "the first band set is the single-image one");
    const bool single = op.n >= kBandMinN && op.bands[0].n_bands > 0;
    op.n_bands = single ? op.bands[0].n_bands : 0;
    op.n_band_order = single ? op.bands[0].n_order : 0;
    op.fb_band_order = single ? op.bands[0].order : nullptr;
    op.n_a_order = int64_t(pl.aorder.size());
    SCT_TRY(lay.take(&op.a_order, 4 * op.n_a_order));
    op.n_orb = int64_t(pl.orbs.size());
    op.a_orb = nullptr;
    if (op.n_orb) SCT_TRY(lay.take(&op.a_orb, int64_t(sizeof(AdjOrbit)) * op.n_orb));
    return RADON_OK;
}

static void op_free(Op *op)
{
    if (!op) return;
    for (void *p : op->owned) (void)hipFree(p);
    delete op;
}

// Owns the hipMalloc'd blocks of build_radon_csr until they are handed to
// the operator (or freed on failure).
struct OwnedBlocks {
    std::vector<void *> ptrs;
    ~OwnedBlocks()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    int alloc(void **p, int64_t bytes)
    {
        *p = nullptr;
        SCT_HIP(hipMalloc(p, size_t(bytes > 0 ? bytes : 256)));
        ptrs.push_back(*p);
        return RADON_OK;
    }
};

}  // namespace sct

using namespace sct;

extern "C" const char *radon_last_error(void) { return sct::last_error(); }

namespace sct {

// Angle runs of one gather class and their groups of op.bang angles (see
// BundleMap), from the measured angles' (cos, sin).
static int bundle_map(Op &op, const std::vector<double> &cs)
{
    BundleMap &m = op.bmap;
    m = BundleMap();
    m.angles = op.bang;
    m.rpa = op.bw / op.bang;
    m.nbpr = (op.n_bins + m.rpa - 1) / m.rpa;
    m.runs = 0;
    int groups = 0;
    const int n_stored = op.sym ? op.n_rep : op.n_meas;   // angles with bundles of their own
    for (int a = 0; a < n_stored;) {
        const bool hz = std::fabs(cs[2 * size_t(a) + 1]) > std::fabs(cs[2 * size_t(a)]);
        int e = a + 1;
        // with one angle per bundle the classes need no runs of their own
        while (e < n_stored &&
               (op.bang == 1 || (std::fabs(cs[2 * size_t(e) + 1]) > std::fabs(cs[2 * size_t(e)])) == hz))
            ++e;
        if (m.runs == kMaxAngleRuns)
            return set_error(RADON_EUNSUPPORTED, "measured angles fall into more than %d runs of one gather class",
                             kMaxAngleRuns);
        m.start[m.runs] = a;
        m.gbase[m.runs] = groups;
        groups += (e - a + op.bang - 1) / op.bang;
        ++m.runs;
        a = e;
    }
    m.start[m.runs] = n_stored;
    m.gbase[m.runs] = groups;
    return RADON_OK;
}

// Storage by the symmetries of the square: the measured angles k (theta =
// pi k / n_angles) with 4k <= n_angles are stored (a prefix of the measured
// list, all closer to vertical); each stands for the measured angles of
// pi - theta, pi/2 - theta and pi/2 + theta that are not itself or an
// earlier partner.  Every measured angle must be stored or such a partner,
// exactly once.
static int symmetry_map(Op &op, const std::vector<double> &cs)
{
    const int na = op.n_angles;
    std::vector<int32_t> pos(size_t(na), -1);   // angle index -> measured position
    for (int a = 0; a < op.n_meas; ++a) pos[size_t(op.meas[size_t(a)])] = a;
    std::vector<int> covered(size_t(op.n_meas), 0);
    op.n_rep = 0;
    op.partner_host.clear();
    for (int a = 0; a < op.n_meas; ++a) {
        const int k = op.meas[size_t(a)];
        if (4 * int64_t(k) > na) break;
        if (std::fabs(cs[2 * size_t(a) + 1]) > std::fabs(cs[2 * size_t(a)]))
            return set_error(RADON_EUNSUPPORTED, "symmetric storage: angle %d of [0, pi/4] is closer to horizontal",
                             k);
        ++op.n_rep;
        ++covered[size_t(a)];
        // partner angle indices in [0, na): pi - theta (none for theta = 0:
        // that is theta itself, with the bins mirrored), pi/2 - theta and
        // pi/2 + theta, which need an even number of angles
        int cand[3] = {k > 0 ? na - k : -1, (na % 2 == 0) ? na / 2 - k : -1, (na % 2 == 0) ? na / 2 + k : -1};
        int got[3] = {-1, -1, -1};
        for (int j = 0; j < 3; ++j) {
            const int c = cand[j];
            if (c < 0 || c >= na || c == k) continue;
            bool dup = false;
            for (int i = 0; i < j; ++i) dup = dup || cand[i] == c;
            if (dup) continue;
            const int pa = pos[size_t(c)];
            if (pa < 0) continue;   // not measured: its rays are not in the operator
            got[j] = pa;
            ++covered[size_t(pa)];
        }
        op.partner_host.push_back(make_int4(got[0], got[1], got[2], -1));
    }
    if (na % 2 != 0) return set_error(RADON_EUNSUPPORTED, "symmetric storage needs an even number of angles");
    for (int a = 0; a < op.n_meas; ++a)
        if (covered[size_t(a)] != 1)
            return set_error(RADON_EUNSUPPORTED,
                             "symmetric storage: measured angle %d is %s (the measured angles must be closed "
                             "under theta -> pi - theta and theta -> pi/2 - theta)",
                             op.meas[size_t(a)], covered[size_t(a)] ? "covered twice" : "not covered");
    return RADON_OK;
}

// Checks the geometry and fills the operator's sizes and angle table (no
// device work).  On success *res owns a new handle without device arrays.
static int new_op(const radon_geom *g, Op **res, std::vector<double> &cs)
{
    *res = nullptr;
    if (!g) return set_error(RADON_EINVAL, "geometry is NULL");
    if (g->n < 1 || g->n > 32767) return set_error(RADON_EINVAL, "n must be in [1, 32767] (got %d)", g->n);
    if (g->n_angles < 1) return set_error(RADON_EINVAL, "n_angles must be >= 1 (got %d)", g->n_angles);
    if (g->n_bins < 1 || g->n_bins > 65535)
        return set_error(RADON_EINVAL, "n_bins must be in [1, 65535] (got %d)", g->n_bins);
    if (g->dtype != SPARSECT_F32 && g->dtype != SPARSECT_F64 && g->dtype != SPARSECT_F32_F64)
        return set_error(RADON_EINVAL, "dtype must be SPARSECT_F32, SPARSECT_F64 or SPARSECT_F32_F64 (got %d)",
                         g->dtype);
    if (g->fwd_bundle != 0 && !valid_bundle_width(g->fwd_bundle))
        return set_error(RADON_EINVAL, "fwd_bundle must be 0, 16, 32 or 64 (got %d)", g->fwd_bundle);
    const int bw = g->fwd_bundle ? g->fwd_bundle : kFwdLanes;
    if (g->fwd_compact != 0 && g->fwd_compact != 1)
        return set_error(RADON_EINVAL, "fwd_compact must be 0 or 1 (got %d)", g->fwd_compact);
    if (g->fwd_symmetric != 0 && g->fwd_symmetric != 1)
        return set_error(RADON_EINVAL, "fwd_symmetric must be 0 or 1 (got %d)", g->fwd_symmetric);
    if (g->fwd_symmetric && g->n < 2) return set_error(RADON_EINVAL, "fwd_symmetric needs n >= 2");
    if (g->fwd_angles != 0 && !valid_bundle_angles(g->fwd_angles, bw))
        return set_error(RADON_EINVAL,
                         "fwd_angles must be 0, 1, 2 or 4 with at least 16 rays per angle "
                         "(got %d angles for a bundle of %d rays)", g->fwd_angles, bw);
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
    op->bw = bw;
    op->bang = g->fwd_angles ? g->fwd_angles : 1;
    op->compact = g->fwd_compact != 0;
    op->sym = g->fwd_symmetric != 0;
    op->tiles = (op->n + 7) / 8;
    op->n_ag = int64_t(op->tiles) * op->tiles;
    op->n_aq = (op->n_meas + 3) / 4;
    op->a_slots = aslots;
    cs.assign(2 * meas.size(), 0.0);
    for (size_t a = 0; a < meas.size(); ++a) {
        angle_cos_sin(meas[a], g->n_angles, &cs[2 * a], &cs[2 * a + 1]);
        if (std::fabs(cs[2 * a + 1]) > std::fabs(cs[2 * a])) op->need_T = true;
    }
    int rc = op->sym ? symmetry_map(*op, cs) : RADON_OK;
    if (rc == RADON_OK) rc = bundle_map(*op, cs);
    if (rc != RADON_OK) {
        delete op;
        return rc;
    }
    // an operator stored by symmetry keeps adjoint slots for its stored
    // angles only when the maps carry whole 8x8 tiles onto tiles
    op->sym_adj = op->sym && op->n % 8 == 0;
    op->n_adj_ang = op->sym_adj ? op->n_rep : op->n_meas;
    op->n_aq = (op->n_adj_ang + 3) / 4;
    op->a_slots = op->n_ag * 64 * 4 * int64_t(op->n_aq);
    op->n_fb = n_fb_of(*op);
    *res = op;
    return RADON_OK;
}

static int fill_typed(Op &op, const Plan &pl, hipStream_t st, const CountTmp &t)
{
    try {
        return op.msize == 4 ? fill_phase<float>(op, pl, st, t) : fill_phase<double>(op, pl, st, t);
    } catch (...) {
        return set_error(RADON_EINVAL, "unexpected host exception during build");
    }
}

static void fill_sizes(const Op &op, const Plan &pl, int64_t ws_need, radon_sizes *out)
{
    out->n_meas_rays = op.rows;
    out->nnz = pl.nnz;
    out->fwd_slots = pl.fslots;
    out->adj_slots = op.a_slots;
    out->row_ptr_bytes = 8 * (op.rows + 1);
    out->col_bytes = 4 * pl.nnz;
    out->val_bytes = int64_t(op.msize) * pl.nnz;
    out->layout_bytes = layout_bytes(op, pl);
    out->ws_bytes = ws_need;
}

}  // namespace sct (host entry helpers)

extern "C" int radon_csr_sizes(const radon_geom *g, void *ws, int64_t ws_bytes, void *stream,
                               radon_sizes *out)
{
    clear_error();
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    std::vector<double> cs;
    Op *op = nullptr;
    SCT_TRY(new_op(g, &op, cs));
    std::unique_ptr<Op> hold(op);
    int64_t need = 0;
    SCT_TRY(build_ws_bytes(*op, &need));
    std::memset(out, 0, sizeof *out);
    out->n_meas_rays = op->rows;
    out->nnz = -1;
    out->ws_bytes = need;
    if (!ws) return RADON_OK;   // query of the workspace size only
    if (ws_bytes < need)
        return set_error(RADON_EWORKSPACE, "radon_csr_sizes needs a workspace of %lld bytes (got %lld)",
                         (long long)need, (long long)ws_bytes);
    if (reinterpret_cast<uintptr_t>(ws) & 255) return set_error(RADON_EINVAL, "ws must be 256-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carve w{static_cast<char *>(ws), ws_bytes, 0, "radon_csr_sizes workspace"};
    int64_t *rp = nullptr;
    FwdBundle *fb = nullptr;
    SCT_TRY(w.take(&rp, 8 * (op->rows + 1)));
    SCT_TRY(w.take(&fb, int64_t(sizeof(FwdBundle)) * op->n_fb));
    CountTmp t;
    Plan pl;
    int rc = count_phase(*op, cs, st, w, rp, fb, t, pl);
    if (rc != RADON_OK) {
        (void)hipStreamSynchronize(st);
        return rc;
    }
    fill_sizes(*op, pl, need, out);
    return RADON_OK;
}

extern "C" int build_radon_csr_into(const radon_geom *g, const radon_buffers *b, void *stream,
                                    radon_op **out)
{
    clear_error();
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    *out = nullptr;
    if (!b) return set_error(RADON_EINVAL, "buffers are NULL");
    std::vector<double> cs;
    Op *op = nullptr;
    SCT_TRY(new_op(g, &op, cs));
    std::unique_ptr<Op> hold(op);
    int64_t need = 0;
    SCT_TRY(build_ws_bytes(*op, &need));
    if (!b->row_ptr || !b->col || !b->val || !b->layout || !b->ws)
        return set_error(RADON_EINVAL, "every buffer of radon_buffers must be non-NULL");
    for (const void *p : {(const void *)b->row_ptr, (const void *)b->col, (const void *)b->val,
                          (const void *)b->layout, (const void *)b->ws})
        if (reinterpret_cast<uintptr_t>(p) & 255)
            return set_error(RADON_EINVAL, "radon_buffers pointers must be 256-byte aligned");
    if (b->ws_bytes < need)
        return set_error(RADON_EWORKSPACE, "build_radon_csr_into needs a workspace of %lld bytes (got %lld)",
                         (long long)need, (long long)b->ws_bytes);
    if (b->row_ptr_bytes < 8 * (op->rows + 1))
        return set_error(RADON_EWORKSPACE, "row_ptr needs %lld bytes (got %lld)",
                         (long long)(8 * (op->rows + 1)), (long long)b->row_ptr_bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carve w{static_cast<char *>(b->ws), b->ws_bytes, 0, "build_radon_csr_into workspace"};
    Carve lay{static_cast<char *>(b->layout), b->layout_bytes, 0, "build_radon_csr_into layout block"};
    // the slots the sizes query uses for the row pointers and bundle table stay unused here
    int64_t *rp_unused = nullptr;
    FwdBundle *fb_unused = nullptr;
    SCT_TRY(w.take(&rp_unused, 8 * (op->rows + 1)));
    SCT_TRY(w.take(&fb_unused, int64_t(sizeof(FwdBundle)) * op->n_fb));
    op->rp = b->row_ptr;
    SCT_TRY(lay.take(&op->fb, int64_t(sizeof(FwdBundle)) * op->n_fb));
    CountTmp t;
    Plan pl;
    int rc = count_phase(*op, cs, st, w, op->rp, op->fb, t, pl);
    if (rc == RADON_OK) {
        op->nnz = pl.nnz;
        op->f_slots = pl.fslots;
        if (b->col_bytes < 4 * pl.nnz || b->val_bytes < int64_t(op->msize) * pl.nnz)
            rc = set_error(RADON_EWORKSPACE, "col and val need %lld and %lld bytes (got %lld and %lld)",
                           (long long)(4 * pl.nnz), (long long)(op->msize * pl.nnz),
                           (long long)b->col_bytes, (long long)b->val_bytes);
    }
    if (rc == RADON_OK) {
        op->col = b->col;
        op->val = b->val;
        rc = carve_layouts(*op, pl, lay, true);
    }
    if (rc == RADON_OK) rc = fill_typed(*op, pl, st, t);
    if (rc != RADON_OK) {
        (void)hipStreamSynchronize(st);
        return rc;
    }
    op->device_bytes = 8 * (op->rows + 1) + 4 * op->nnz + int64_t(op->msize) * op->nnz + lay.used;
    *out = reinterpret_cast<radon_op *>(hold.release());
    return RADON_OK;
}

extern "C" int build_radon_csr(const radon_geom *g, void *stream, radon_op **out)
{
    clear_error();
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    *out = nullptr;
    std::vector<double> cs;
    Op *op = nullptr;
    SCT_TRY(new_op(g, &op, cs));
    std::unique_ptr<Op, void (*)(Op *)> hold(op, op_free);
    int64_t need = 0;
    SCT_TRY(build_ws_bytes(*op, &need));
    hipStream_t st = static_cast<hipStream_t>(stream);
    OwnedBlocks tmp, keep;
    void *wsp = nullptr, *rp = nullptr, *fbp = nullptr;
    SCT_TRY(tmp.alloc(&wsp, need));
    SCT_TRY(keep.alloc(&rp, 8 * (op->rows + 1)));
    SCT_TRY(keep.alloc(&fbp, int64_t(sizeof(FwdBundle)) * op->n_fb));
    Carve w{static_cast<char *>(wsp), need, 0, "build_radon_csr workspace"};
    int64_t *rp_unused = nullptr;
    FwdBundle *fb_unused = nullptr;
    SCT_TRY(w.take(&rp_unused, 8 * (op->rows + 1)));
    SCT_TRY(w.take(&fb_unused, int64_t(sizeof(FwdBundle)) * op->n_fb));
    op->rp = static_cast<int64_t *>(rp);
    op->fb = static_cast<FwdBundle *>(fbp);
    CountTmp t;
    Plan pl;
    int rc = count_phase(*op, cs, st, w, op->rp, op->fb, t, pl);
    void *col = nullptr, *val = nullptr, *layp = nullptr;
    int64_t lb = 0;
    if (rc == RADON_OK) {
        op->nnz = pl.nnz;
        op->f_slots = pl.fslots;
        lb = layout_bytes(*op, pl);
        rc = keep.alloc(&col, 4 * pl.nnz);
        if (rc == RADON_OK) rc = keep.alloc(&val, int64_t(op->msize) * pl.nnz);
        if (rc == RADON_OK) rc = keep.alloc(&layp, lb);
    }
    if (rc == RADON_OK) {
        op->col = static_cast<int32_t *>(col);
        op->val = val;
        // the bundle table has its own block here: its room at the start of
        // the layout block stays unused
        Carve lay{static_cast<char *>(layp), lb, 0, "build_radon_csr layout block"};
        FwdBundle *fb_room = nullptr;
        rc = lay.take(&fb_room, int64_t(sizeof(FwdBundle)) * op->n_fb);
        if (rc == RADON_OK) rc = carve_layouts(*op, pl, lay, true);
    }
    if (rc == RADON_OK) rc = fill_typed(*op, pl, st, t);
    if (rc != RADON_OK) {
        (void)hipStreamSynchronize(st);
        return rc;
    }
    op->owned = keep.ptrs;
    keep.ptrs.clear();
    op->device_bytes = 8 * (op->rows + 1) + int64_t(sizeof(FwdBundle)) * op->n_fb + 4 * op->nnz +
                       int64_t(op->msize) * op->nnz + lb;
    *out = reinterpret_cast<radon_op *>(hold.release());
    return RADON_OK;
}

static_assert(sizeof(radon_geom) == 40 && sizeof(radon_info) == 104, "C ABI struct sizes");

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
    out->fwd_bundle = op->bw;
    out->fwd_angles = op->bang;
    out->fwd_compact = op->compact ? 1 : 0;
    out->fwd_symmetric = op->sym ? 1 : 0;
    out->adj_symmetric = op->sym_adj ? 1 : 0;
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
    // measured angle -> (angle with slots, map): an adjoint stored by
    // symmetry holds the records of a partner angle at the stored angle, for
    // the pixel's image under the inverse map (see k_adj1_sym)
    std::vector<int2> src(size_t(op.n_meas));
    for (int a = 0; a < op.n_meas; ++a) src[size_t(a)] = make_int2(a, 0);
    if (op.sym_adj)
        for (int a = 0; a < op.n_rep; ++a) {
            const int4 p = op.partner_host[size_t(a)];
            const int pm[3] = {p.x, p.y, p.z};
            for (int mu = 1; mu <= 3; ++mu)
                if (pm[mu - 1] >= 0) src[size_t(pm[mu - 1])] = make_int2(a, mu);
        }
    const int n = op.n;
    for (int64_t j = 0; j < op.nn; ++j)
        for (int a = 0; a < op.n_meas; ++a) {
            const int px = int(j % n), py = int(j / n), mu = src[size_t(a)].y;
            const int qx = mu == 0 ? px : (mu == 1 ? n - 1 - px : py);
            const int qy = mu == 0 ? py : (mu == 1 ? py : (mu == 2 ? px : n - 1 - px));
            const size_t s = size_t(adj_slot(qy, qx, src[size_t(a)].x, op.n_aq, op.tiles));
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
