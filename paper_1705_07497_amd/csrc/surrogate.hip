// Surrogate operator T of Section 3.2 (eq:def_sparse_surr, eq:surr_SBupd).
//
// T is the sum over all pixels q of the centre pixel's point-spread function
// P = R^T M^T M R e_c moved to q and cut to the disc of radius r around q,
// with the entries that fall outside the image dropped (the paper suppresses
// the wrap-around to the opposite edge).  Here the weights come from this
// operator's own products (one forward and one adjoint of e_c) and T is
// taken as the symmetric part of that sum, w(d) = (P_{c+d} + P_{c-d}) / 2,
// because the surrogate system is solved by CG.  Applying T is a
// (2r+1)^2-point stencil: an HBM-bound pass over the image, no matrix.
#include "cg.hpp"
#include "products.hpp"

#include <cmath>
#include <new>

namespace sct {

constexpr int kSurMaxR = 8;   // LDS tile of (32 + 2r)^2 values

// out = alpha (T x) + lambda (K^T K x) + sigma x on one 32x32 tile per block
// (32 x 8 threads, 4 rows each) with the tile and a halo of max(r, 1) staged
// in LDS; the FP64 partial <x, out> of the tile goes to part.
template <class T>
__global__ __launch_bounds__(256) void k_stencil(const T *__restrict__ x, T *__restrict__ out,
                                                 const T *__restrict__ wts, int r, T alpha,
                                                 T lambda, T sigma, double *__restrict__ part,
                                                 int n, int64_t nn)
{
    constexpr int kMax = 32 + 2 * kSurMaxR;
    __shared__ T tile[kMax][kMax + 1];
    __shared__ T ws[(2 * kSurMaxR + 1) * (2 * kSurMaxR + 1)];
    __shared__ double red[256];
    const int h = r > 1 ? r : 1;
    const int side = 32 + 2 * h, k = 2 * r + 1;
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int64_t off = int64_t(blockIdx.z) * nn;
    const int t = threadIdx.y * 32 + threadIdx.x;
    for (int i = t; i < k * k; i += 256) ws[i] = wts[i];
    for (int i = t; i < side * side; i += 256) {
        const int ly = i / side, lx = i % side;
        const int gy = by + ly - h, gx = bx + lx - h;
        tile[ly][lx] = (gy >= 0 && gy < n && gx >= 0 && gx < n) ? x[off + int64_t(gy) * n + gx] : T(0);
    }
    __syncthreads();
    double acc_dot = 0.0;
    for (int i = threadIdx.y; i < 32; i += 8) {
        const int py = by + i, px = bx + threadIdx.x;
        if (py >= n || px >= n) continue;
        const int ly = i + h, lx = threadIdx.x + h;
        // (T x)_p = sum_d w(d) x_{p - d}, out-of-image taps read the zero halo
        T tx = T(0);
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx)
                tx = fma(ws[(dy + r) * k + (dx + r)], tile[ly - dy][lx - dx], tx);
        const T xj = tile[ly][lx];
        T o = alpha * tx;
        if (lambda != T(0)) {
            T ktk = T(0);   // Neumann 5-point K^T K, as in the normal operator
            if (px > 0) ktk += xj - tile[ly][lx - 1];
            if (px < n - 1) ktk += xj - tile[ly][lx + 1];
            if (py > 0) ktk += xj - tile[ly - 1][lx];
            if (py < n - 1) ktk += xj - tile[ly + 1][lx];
            o += lambda * ktk;
        }
        if (sigma != T(0)) o += sigma * xj;
        out[off + int64_t(py) * n + px] = o;
        acc_dot += double(xj) * double(o);
    }
    if (!part) return;
    const double tot = block_sum(acc_dot, red);
    if (t == 0)
        part[int64_t(blockIdx.z) * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = tot;
}

int64_t surrogate_parts(const Sur &s)
{
    const int64_t t = tiles_of(s.n);
    return t * t;
}

template <class TV>
int launch_surrogate(const Sur &s, double alpha, double lambda, double sigma, const TV *x, TV *out,
                     double *part, int batch, hipStream_t st)
{
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    const unsigned t = unsigned(tiles_of(s.n));
    k_stencil<TV><<<dim3(t, t, unsigned(batch)), dim3(32, 8), 0, st>>>(
        x, out, static_cast<const TV *>(s.w_dev), s.r, TV(alpha), TV(lambda), TV(sigma), part, s.n,
        s.nn);
    return check_launch("k_stencil");
}

template int launch_surrogate<float>(const Sur &, double, double, double, const float *, float *,
                                     double *, int, hipStream_t);
template int launch_surrogate<double>(const Sur &, double, double, double, const double *, double *,
                                      double *, int, hipStream_t);

template <class TV>
__global__ void k_unit(TV *__restrict__ e, int64_t j)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) e[j] = TV(1);
}

// P = R^T M^T M R e_c (device), window of radius r copied to the host.
template <class TM, class TV>
static int surrogate_psf(const Op &op, int r, std::vector<double> &win, hipStream_t st)
{
    const int n = op.n, c = n / 2, k = 2 * r + 1;
    std::vector<void *> tmp;
    auto cleanup = [&]() {
        for (void *p : tmp) (void)hipFree(p);
    };
    auto alloc = [&](void **p, int64_t bytes) -> int {
        *p = nullptr;
        const hipError_t e = hipMalloc(p, size_t(bytes > 0 ? bytes : 256));
        if (e != hipSuccess) return set_error(RADON_EHIP, "hipMalloc failed: %s", hipGetErrorString(e));
        tmp.push_back(*p);
        return RADON_OK;
    };
    TV *e = nullptr, *eT = nullptr, *y = nullptr, *P = nullptr;
    int rc = alloc(reinterpret_cast<void **>(&e), int64_t(sizeof(TV)) * op.nn);
    if (rc == RADON_OK && op.need_T) rc = alloc(reinterpret_cast<void **>(&eT), int64_t(sizeof(TV)) * op.nn);
    if (rc == RADON_OK) rc = alloc(reinterpret_cast<void **>(&y), int64_t(sizeof(TV)) * op.rows);
    if (rc == RADON_OK) rc = alloc(reinterpret_cast<void **>(&P), int64_t(sizeof(TV)) * op.nn);
    if (rc != RADON_OK) {
        cleanup();
        return rc;
    }
    const int64_t jc = int64_t(c) * n + c;
    std::vector<TV> rowbuf(static_cast<size_t>(k));
    hipError_t he = hipMemsetAsync(e, 0, sizeof(TV) * size_t(op.nn), st);
    if (he == hipSuccess) {
        k_unit<TV><<<1, 64, 0, st>>>(e, jc);
        rc = check_launch("k_unit");
        if (rc == RADON_OK && eT) rc = launch_transpose<TV>(op, e, eT, 1, st);
        if (rc == RADON_OK) rc = launch_fwd<TM, TV>(op, e, eT, y, 1, st);
        if (rc == RADON_OK) rc = launch_adj<TM, TV>(op, y, nullptr, P, 1.0, 0.0, 0.0, nullptr, 1, st);
        if (rc == RADON_OK) he = hipStreamSynchronize(st);
        for (int dy = -r; rc == RADON_OK && he == hipSuccess && dy <= r; ++dy) {
            he = hipMemcpy(rowbuf.data(), P + int64_t(c + dy) * n + (c - r), sizeof(TV) * size_t(k),
                           hipMemcpyDeviceToHost);
            for (int i = 0; i < k; ++i) win[size_t((dy + r) * k + i)] = double(rowbuf[size_t(i)]);
        }
    }
    cleanup();
    if (rc != RADON_OK) return rc;
    if (he != hipSuccess) return set_error(RADON_EHIP, "surrogate build: %s", hipGetErrorString(he));
    return RADON_OK;
}

static void free_sur(Sur *s)
{
    if (!s) return;
    if (s->w_dev) (void)hipFree(s->w_dev);
    delete s;
}

}  // namespace sct

using namespace sct;

extern "C" int radon_surrogate_create(const radon_op *p, int32_t radius, void *stream,
                                      radon_surrogate **out)
{
    clear_error();
    if (!out) return set_error(RADON_EINVAL, "out is NULL");
    *out = nullptr;
    SCT_TRY(check_op(p));
    const Op &op = *as_op(p);
    const int n = op.n, c = n / 2;
    if (radius < 0 || radius > kSurMaxR)
        return set_error(RADON_EINVAL, "radius must be in [0, %d] (got %d)", kSurMaxR, radius);
    if (c - radius < 0 || c + radius >= n)
        return set_error(RADON_EINVAL, "the disc of radius %d around pixel (%d, %d) leaves the image",
                         radius, c, c);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int k = 2 * radius + 1;
    std::vector<double> win(size_t(k * k), 0.0);
    SCT_TRY(dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        return surrogate_psf<TM, TV>(op, radius, win, st);
    }));
    Sur *s = new (std::nothrow) Sur;
    if (!s) return set_error(RADON_EINVAL, "out of host memory");
    s->n = n;
    s->nn = op.nn;
    s->r = radius;
    s->dtype = op.dtype;
    s->vsize = op.vsize;
    s->w.assign(size_t(k * k), 0.0);
    for (int dy = -radius; dy <= radius; ++dy)
        for (int dx = -radius; dx <= radius; ++dx)
            if (dy * dy + dx * dx <= radius * radius)
                s->w[size_t((dy + radius) * k + dx + radius)] =
                    0.5 * (win[size_t((dy + radius) * k + dx + radius)] +
                           win[size_t((radius - dy) * k + radius - dx)]);
    hipError_t e = hipMalloc(&s->w_dev, size_t(s->vsize) * size_t(k * k));
    if (e == hipSuccess) {
        if (s->vsize == 4) {
            std::vector<float> wf(s->w.begin(), s->w.end());
            e = hipMemcpy(s->w_dev, wf.data(), 4 * wf.size(), hipMemcpyHostToDevice);
        } else {
            e = hipMemcpy(s->w_dev, s->w.data(), 8 * s->w.size(), hipMemcpyHostToDevice);
        }
    }
    if (e != hipSuccess) {
        free_sur(s);
        return set_error(RADON_EHIP, "surrogate weights: %s", hipGetErrorString(e));
    }
    *out = reinterpret_cast<radon_surrogate *>(s);
    return RADON_OK;
}

extern "C" void radon_surrogate_destroy(radon_surrogate *s) { free_sur(reinterpret_cast<Sur *>(s)); }

extern "C" int radon_surrogate_weights(const radon_surrogate *p, int32_t *radius, double *w)
{
    clear_error();
    if (!p) return set_error(RADON_EINVAL, "surrogate is NULL");
    const Sur &s = *reinterpret_cast<const Sur *>(p);
    if (radius) *radius = s.r;
    if (w)
        for (size_t i = 0; i < s.w.size(); ++i) w[i] = s.w[i];
    return RADON_OK;
}

extern "C" int surrogate_apply(const radon_surrogate *p, double alpha, double lambda, double sigma,
                               const void *x, void *out, double *dot_out, int32_t batch,
                               void *ws, int64_t ws_bytes, void *stream)
{
    clear_error();
    if (!p) return set_error(RADON_EINVAL, "surrogate is NULL");
    SCT_TRY(check_batch(batch));
    if (!x || !out) return set_error(RADON_EINVAL, "x and out must be non-NULL");
    if (x == out) return set_error(RADON_EINVAL, "out must not alias x");
    const Sur &s = *reinterpret_cast<const Sur *>(p);
    const int64_t need = dot_out ? int64_t(8) * surrogate_parts(s) * batch : 0;
    SCT_TRY(check_ws(ws, ws_bytes, need, "surrogate_apply"));
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *part = dot_out ? static_cast<double *>(ws) : nullptr;
    if (s.vsize == 4)
        SCT_TRY(launch_surrogate<float>(s, alpha, lambda, sigma, static_cast<const float *>(x),
                                        static_cast<float *>(out), part, batch, st));
    else
        SCT_TRY(launch_surrogate<double>(s, alpha, lambda, sigma, static_cast<const double *>(x),
                                         static_cast<double *>(out), part, batch, st));
    if (dot_out) SCT_TRY(launch_sum_partials(part, surrogate_parts(s), dot_out, batch, st));
    return RADON_OK;
}
