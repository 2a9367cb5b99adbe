// Internal declarations of the sparsect library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/sparsect.h"

namespace sct {

// Forward product layout: one bundle = up to R adjacent bins of each of up to
// A consecutive measured angles of one gather class (A, the angles per
// bundle, is 1, 2 or 4; BW = A*R, the bundle width, is 16, 32 or 64; both are
// chosen when the operator is built).  Lane r of a bundle is angle r / R, bin
// r % R.  Slot (t, r) covers lane r's ray on image line m0 + t along the
// rays' major axis (rows for rays closer to vertical, columns for rays closer
// to horizontal): the first of the (at most two adjacent) pixels the ray
// meets on that line, the ray's length in it and its length in the second.
// A compact operator does not store the second length: on a line the ray
// crosses from one side to the other the two lengths add up to the same
// chord on every such line (1/|cos| or 1/|sin| of the angle), so the second
// is that chord minus the first; only the ray's first and last lines can be
// crossed in part (where it enters or leaves the image), and their second
// lengths are kept per ray (RayEdge).  Its forward then uses, for the FP32
// matrix, second lengths within about one FP32 rounding of the chord of the
// stored (CSR) ones; the CSR and the adjoint keep the stored values.
// Slots are grouped in quads of 4 consecutive lines of one ray so that a
// lane reads 4 slots with one 16-byte load:
//   slot(t, r) = off + ((t/4)*BW + r)*4 + t%4.
// A wave's 64 lanes cover BW rays and 64/BW consecutive quads, so one gather
// instruction reads the BW rays on each of 64/BW image lines.  The rays of
// neighbouring angles and the same bins cross an image line a few pixels
// apart, so with A > 1 the lanes of one gather share most of their cache
// lines.
constexpr int kFwdLanes = 16;   // default bundle width
inline bool valid_bundle_width(int bw) { return bw == 16 || bw == 32 || bw == 64; }
inline bool valid_bundle_angles(int a, int bw) { return (a == 1 || a == 2 || a == 4) && bw / a >= 16; }
// Adjoint layout: one group = an 8x8 pixel tile (tile (ty, tx) is group
// g = ty*tiles + tx, tiles = ceil(n/8); lane l = (iy%8)*8 + ix%8), chosen
// because an 8x8 tile projects onto at most 14 adjacent bins at any angle, so
// the 64 lanes' sinogram gathers hit one or two cache lines.  Slot (a, l)
// covers the lane's pixel at measured angle a; quads of 4 consecutive angles
// of one pixel are contiguous:
//   slot(g, l, a) = ((g*nq + a/4)*64 + l)*4 + a%4,
// with nq = ceil(n_meas/4) (angles past n_meas in the last quad are zero;
// lanes outside the image are zero too).  A slot stores its first bin as an
// 8-bit offset from the tile's lowest bin at that angle (the tile's bins span
// at most 13, so bin and bin+1 fall in a 16-bin band starting at the base).
constexpr int kAdjLanes = 64;
// Line bands of the forward product: 128 lines of a 1024- or 2048-pixel FP64
// image are 1 or 2 MB of an XCD's 4 MB L2.  Images from 1024 pixels on (8 MB
// and more per gather class) use them; at 512 the whole image already stays
// in L2 and the bands only add work (measured on the 512 x 512, 1024 x 1024
// and 2048 x 2048 operators; 64- and 256-line bands were slower).
constexpr int kBandLines = 128;
constexpr int kBandMinN = 1024;
constexpr int kAdjBand = 16;
// Fused multi-image forwards gather from every image of their chunk, so the
// band that stays in an XCD's L2 is the chunk's images' band together: the
// band height is the largest of these whose chunk band fits the budget.
constexpr int kBandHeights[4] = {128, 64, 32, 16};
constexpr int64_t kBandBudget = int64_t(2) << 20;
constexpr int kBandSetMinN = 256;   // band sets are built from this image side on

// One band height's work list of the line-banded forward.
struct BandSet {
    int32_t lines = 0, n_bands = 0;
    int2 *order = nullptr;           // (bundle, band), padding (-1, -1)
    int64_t n_order = 0;
};

__host__ __device__ inline int64_t fwd_slot(int64_t off, int t, int r, int bw)
{
    return off + ((int64_t(t >> 2) * bw + r) << 2) + (t & 3);
}

__host__ __device__ inline int64_t adj_slot(int iy, int ix, int a, int nq, int tiles)
{
    const int64_t g = int64_t(iy >> 3) * tiles + (ix >> 3);
    const int l = ((iy & 7) << 3) | (ix & 7);
    return (((g * nq + (a >> 2)) * kAdjLanes + l) << 2) + (a & 3);
}

struct FwdBundle {
    int64_t off;      // first slot
    int32_t m0;       // first major line
    int32_t nrows;    // major lines covered (multiple of 4, may be 0)
    int32_t ray0;     // measured ray of lane 0 (first angle, first bin)
    int32_t astride;  // measured rays from one angle of the bundle to the next (n_bins)
    int16_t nrays;    // bins per angle in the bundle (<= R)
    int16_t nang;     // angles in the bundle (<= A)
    int16_t rshift;   // log2 R: lane r is angle r >> rshift, bin r & (R - 1)
    int16_t horiz;    // 1: major axis is x (gather from the transposed image)
};
static_assert(sizeof(FwdBundle) == 32, "FwdBundle layout");

// Per measured ray: its chord on a fully crossed major line (the sum of its
// two lengths there, from the build's own lengths), its first and last major
// lines and the second lengths on those two (rounded to the matrix type).  A
// ray without pixels has mf > ml.
struct RayEdge {
    double chord, w1f, w1l;
    int32_t mf, ml;
};
static_assert(sizeof(RayEdge) == 32, "RayEdge layout");

// One orbit of 8x8 tiles under x -> -x and the transpose, for an adjoint
// stored by symmetry: its tiles (-1 past the orbit's 1, 4 or 8), and for
// output tile t and map m (identity, x -> -x, transpose, both) the place in
// `tile` of the source tile whose slots feed it under that map.
struct AdjOrbit {
    int32_t tile[8];
    uint8_t src[8][4];
};
static_assert(sizeof(AdjOrbit) == 64, "AdjOrbit layout");

// Measured ray of lane r of bundle d, or -1 for a lane without a ray.
__host__ __device__ inline int64_t bundle_ray(const FwdBundle &d, int r)
{
    const int j = r >> d.rshift, k = r & ((1 << d.rshift) - 1);
    if (j >= d.nang || k >= d.nrays) return -1;
    return int64_t(d.ray0) + int64_t(j) * d.astride + k;
}

// Angles -> bundles.  The measured angles (in index order) fall into runs of
// one gather class (at most three: up to pi/4, to 3pi/4, to pi); each run is
// cut into groups of A consecutive angles, group g holding bundles
// g*nbpr .. g*nbpr + nbpr - 1 of R bins each (nbpr = ceil(n_bins / R)).
constexpr int kMaxAngleRuns = 4;
struct BundleMap {
    int32_t angles = 1, rpa = kFwdLanes, nbpr = 0, runs = 1;
    int32_t start[kMaxAngleRuns + 1] = {};   // first measured angle of each run; start[runs] = n_meas
    int32_t gbase[kMaxAngleRuns + 1] = {};   // first group of each run; gbase[runs] = groups

    __host__ __device__ int64_t bundles() const { return int64_t(gbase[runs]) * nbpr; }
    // bundle of (measured angle a, bin) and the ray's lane in it
    __host__ __device__ int64_t bundle_of(int a, int bin, int *lane) const
    {
        int k = 0;
        while (k + 1 < runs && a >= start[k + 1]) ++k;
        const int rel = a - start[k];
        *lane = (rel % angles) * rpa + bin % rpa;
        return int64_t(gbase[k] + rel / angles) * nbpr + bin / rpa;
    }
    // first measured angle and angle count of group g
    __host__ __device__ void group(int64_t g, int *a0, int *na) const
    {
        int k = 0;
        while (k + 1 < runs && g >= gbase[k + 1]) ++k;
        *a0 = start[k] + int(g - gbase[k]) * angles;
        const int left = start[k + 1] - *a0;
        *na = left < angles ? left : angles;
    }
};

struct Op {
    int32_t n = 0, n_angles = 0, n_bins = 0, dtype = 0;
    int32_t n_meas = 0;              // measured angles
    int64_t nn = 0;                  // pixels
    int64_t rows = 0;                // measured rays
    int64_t nnz = 0;
    bool need_T = false;             // some measured angle uses the transposed image
    std::vector<int32_t> meas;       // measured angle indices (host)
    int32_t msize = 4;               // bytes per stored matrix value
    int32_t vsize = 4;               // bytes per vector element
    int32_t bw = kFwdLanes;          // lanes (rays) per forward bundle (16, 32 or 64)
    int32_t bang = 1;                // measured angles per forward bundle (1, 2 or 4)
    BundleMap bmap;                  // angles -> forward bundles

    // CSR of MR (device)
    int64_t *rp = nullptr;
    int32_t *col = nullptr;
    void *val = nullptr;

    // forward ray-bundle layout (device)
    int64_t n_fb = 0, f_slots = 0;
    FwdBundle *fb = nullptr;
    int32_t *fb_order = nullptr;     // block -> bundle (-1: idle), XCD-aware
    int64_t n_order = 0;
    uint16_t *f_idx = nullptr;
    bool compact = false;            // forward derives the second lengths (no f_v1)
    // stored by the symmetries of the square: bundles only for the first
    // n_rep measured angles (theta in [0, pi/4]), each ray also standing for
    // the rays of f_partner[a] (see fwd_sym.hpp)
    bool sym = false;
    int32_t n_rep = 0;
    // the adjoint stored by symmetry too (n a multiple of 8, so the maps
    // carry 8x8 tiles onto tiles): pixel-group slots for the first n_rep
    // angles only; n_adj_ang is the number of angles with adjoint slots
    bool sym_adj = false;
    int32_t n_adj_ang = 0;
    std::vector<int4> partner_host;
    int4 *f_partner = nullptr;
    void *f_v0 = nullptr;            // first lengths, per slot
    void *f_v1 = nullptr;            // second lengths, per slot (nullptr when compact)
    RayEdge *f_edge = nullptr;       // per measured ray

    // adjoint pixel-group layout (device)
    int64_t n_ag = 0, a_slots = 0;
    int32_t n_aq = 0;                // angle quads per pixel: ceil(n_meas / 4)
    int32_t tiles = 0;               // 8x8 tiles per image side: ceil(n / 8)
    uint16_t *a_base = nullptr;      // [n_ag][n_aq][4]: lowest bin the tile meets at each angle
    uint8_t *a_rel = nullptr;        // per slot: first bin of the pixel minus the tile's base
    void *a_v0 = nullptr, *a_v1 = nullptr;

    int64_t device_bytes = 0;
    std::vector<void *> owned;       // every hipMalloc of the handle

    // line bands of the forward product for images larger than an XCD's L2:
    // work items (bundle, band) in band-major order per XCD, one partial sum
    // per band and ray, added in band order by k_fwd_band_sum.  bands[i] has
    // kBandHeights[i] lines; the single-image path and the group use the
    // 128-line set (n_bands > 0 from kBandMinN on), fused chunks the height
    // their chunk fits.
    BandSet bands[4];
    int32_t n_bands = 0;             // 0: no banded single-image path
    int2 *fb_band_order = nullptr;   // = bands[0].order when n_bands > 0
    int64_t n_band_order = 0;

    // adjoint tile order of the fused multi-image product: the tiles in Morton
    // order cut into 8 runs, run x taken by the workgroups on XCD x, so each
    // XCD's concurrently active tiles form a compact region whose sinogram
    // bands stay in its L2; entries -1 pad each run
    int32_t *a_order = nullptr;
    int64_t n_a_order = 0;
    AdjOrbit *a_orb = nullptr;   // sym_adj: the tile orbits (k_adj1_orb)
    int64_t n_orb = 0;

    radon_tuning tune{2, 0, 4, 8, 0, 0, 0, 0};   // launch tuning (see radon_set_tuning)
};

// thread-local error state
int set_error(int code, const char *fmt, ...);
void clear_error();

#define SCT_HIP(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return ::sct::set_error(RADON_EHIP, "%s failed: %s", #expr,              \
                                    hipGetErrorString(e_));                           \
    } while (0)

#define SCT_TRY(...)                                                                  \
    do {                                                                              \
        int s_ = (__VA_ARGS__);                                                       \
        if (s_ != RADON_OK) return s_;                                                \
    } while (0)

inline int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(RADON_EHIP, "launch of %s failed: %s", what, hipGetErrorString(e));
    return RADON_OK;
}

inline const Op *as_op(const radon_op *p) { return reinterpret_cast<const Op *>(p); }
inline Op *as_op(radon_op *p) { return reinterpret_cast<Op *>(p); }

int check_op(const radon_op *p);
int check_batch(int32_t batch);
int check_ws(const void *ws, int64_t ws_bytes, int64_t need, const char *what);

// Workspace carving: 256-byte aligned sub-buffers.
struct Carver {
    char *base;
    int64_t used = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(int64_t count)
    {
        used = (used + 255) & ~int64_t(255);
        T *p = reinterpret_cast<T *>(base ? base + used : nullptr);
        used += count * int64_t(sizeof(T));
        return p;
    }
};

// Calls f(TM*, TV*) with null pointers whose types name the operator's matrix
// value type TM and vector type TV.
template <class F>
int dispatch(const Op &op, F &&f)
{
    switch (op.dtype) {
    case SPARSECT_F32: return f(static_cast<float *>(nullptr), static_cast<float *>(nullptr));
    case SPARSECT_F64: return f(static_cast<double *>(nullptr), static_cast<double *>(nullptr));
    default: return f(static_cast<float *>(nullptr), static_cast<double *>(nullptr));
    }
}
#define SCT_TYPES(tm, tv)                                 \
    using TM = std::remove_pointer_t<decltype(tm)>;       \
    using TV = std::remove_pointer_t<decltype(tv)>

// --- apply-level launchers (apply.hip) ----------------------------------------
// Transposed copy of `batch` n x n images.
template <class TV>
int launch_transpose(const Op &op, const TV *x, TV *xT, int batch, hipStream_t s);
// y = MR x, gathering from x and (for horizontal bundles) xT.
// With part (fwd_part_elems(op, batch) elements) the forward runs line-banded
// when the operator has bands.
template <class TM, class TV>
int launch_fwd(const Op &op, const TV *x, const TV *xT, TV *y, int batch, hipStream_t s,
               TV *part = nullptr);
// launch_fwd for operators of bundle width BW (fwd16.hip, fwd32.hip, fwd64.hip).
template <class TM, class TV, int BW>
int launch_fwd_bw(const Op &op, const TV *x, const TV *xT, TV *y, int batch, hipStream_t s,
                  TV *part);
// Scratch elements of a forward over `batch` images that has a workspace (0:
// none needed): one chunk's band partials and, for the pixel-major gather
// layout, the chunk's pixel-major copies; the chunks run one after another.
int64_t fwd_part_elems(const Op &op, int batch);
// The same for a chunk of bc images (nb of them present) under a given
// gather layout and band height (tuning values).
int64_t fwd_scratch_elems(const Op &op, int bc, int nb, int layout, int lines);
// Images sharing each matrix load in a forward over `batch` images.
int fwd_chunk(const Op &op, int batch);
// The band set of a forward over chunks of bc images at band height `lines`
// (0: the budget rule), or nullptr when the chunk's whole images fit the
// budget (or the operator has no bands).
const BandSet *band_set_lines(const Op &op, int bc, int lines);
inline const BandSet *band_set_for(const Op &op, int bc) { return band_set_lines(op, bc, op.tune.fwd_lines); }
// Whether a forward chunk of bc images gathers from a pixel-major copy.
inline bool fwd_pixel_major(int layout, int bc) { return layout == 1 && bc >= 4; }
// Elements of alignment slack before a pixel-major copy in the scratch.
constexpr int64_t kPixelMajorSlack = 64;
// Ticket counters of work handed out in list order: one per XCD, each on its
// own 256-byte line (device-scope atomics on one line serialize at one
// channel).
constexpr int kTicketStride = 64;
constexpr int64_t kTicketBytes = 4 * 8 * kTicketStride;
// Scratch elements (of 4 bytes or more) that hold the banded forward's ticket
// counters after its partials, 256-byte aligned.
constexpr int64_t kTicketSlack = (kTicketBytes + 256) / 4;
// A forward chunk's scratch: band partials (part_elems), then the ticket
// counters at the next 256-byte boundary, then the pixel-major copies.
template <class TV>
inline void fwd_scratch_layout(TV *part, int64_t part_elems, uint32_t **tickets, TV **xp)
{
    const uintptr_t a = (reinterpret_cast<uintptr_t>(part + part_elems) + 255) & ~uintptr_t(255);
    *tickets = reinterpret_cast<uint32_t *>(a);
    *xp = reinterpret_cast<TV *>(a + kTicketBytes);
}
// out = alpha (MR)^T y + lambda K^T K x + sigma x; partial <x, out> per group
// into part[batch][n_ag] when part != nullptr.  x may be nullptr when
// lambda == sigma == 0 and part == nullptr.  With scratch
// (adj_scratch_elems(op, batch) elements) a chunk stages its bands from a
// pixel-major copy of its sinograms when the tuning asks for it.
template <class TM, class TV>
int launch_adj(const Op &op, const TV *y, const TV *x, TV *out, double alpha, double lambda,
               double sigma, double *part, int batch, hipStream_t s, TV *scratch = nullptr);
// Scratch elements of a fused adjoint over `batch` sinograms (0: none).
int64_t adj_scratch_elems(const Op &op, int batch);
// Scratch of a normal-operator product (the forward's, then the adjoint's,
// in one region: the adjoint starts after the forward has finished with it).
int64_t prod_scratch_elems(const Op &op, int batch);
// Batched vectors at the C ABI come in RADON_LAYOUT_IMAGE ([batch][count])
// or RADON_LAYOUT_PIXEL ([count][batch]); the kernels work on the former, so
// a pixel-major call relays its inputs and outputs through its workspace.
int check_layout(int32_t layout);
// dst = src between [batch][count] and [count][batch] (to_pixel: from the
// former to the latter), through 32 x 32 tiles in LDS.
template <class TV>
int launch_relayout(const TV *src, TV *dst, int64_t count, int batch, bool to_pixel, hipStream_t s);
// Bytes a pixel-major call of workspace kind `which` needs after the
// image-major workspace (0 for batch 1, where both layouts are one).
int64_t pixel_layout_extra(const Op &op, int which, int batch);
// The two relay buffers of a pixel-major call (n0 and n1 elements), 256-byte
// aligned after the first `base` bytes of ws.
template <class TV>
void relay_buffers(void *ws, int64_t base, int64_t n0, int64_t n1, TV **b0, TV **b1);
// Whether a call relays: pixel-major with more than one image.
inline bool relays(int32_t layout, int batch) { return layout == RADON_LAYOUT_PIXEL && batch > 1; }
// Persistent product kernels use a fixed grid of 8 workgroups per CU (256 CUs)
// that loop over the work items; the adjoint leaves one <x, out> partial per
// workgroup, adj_blocks(op) of them per right-hand side.
constexpr int kPersistentBlocks = 2048;
// Waves per 8x8 tile of the adjoint when the operator's tuning leaves it open:
// two once there are enough measured-angle quads to split (measured on the
// 512 x 512 / 180-angle, 512 x 512 / 120-angle and 1024 x 1024 / 360-angle
// operators, 2 beats 1 and 4).
inline int adj_waves_for(int n_meas) { return n_meas >= 48 ? 2 : 1; }
int adj_blocks(const Op &op);

// Surrogate operator T of Section 3.2 (surrogate.hip): a translated stencil of
// radius r over the image, weights w[(dy + r)(2r + 1) + dx + r].
struct Sur {
    int32_t n = 0, r = 0, dtype = 0, vsize = 4;
    int64_t nn = 0;
    std::vector<double> w;     // host copy of the weights
    void *w_dev = nullptr;     // weights in the vector type
};
// out = alpha T x + lambda K^T K x + sigma x for `batch` images; partial
// <x, out> per 32x32 tile into part[batch][surrogate_parts] when part != nullptr.
template <class TV>
int launch_surrogate(const Sur &s, double alpha, double lambda, double sigma, const TV *x, TV *out,
                     double *part, int batch, hipStream_t st);
int64_t surrogate_parts(const Sur &s);

// Fourier-domain operator of Sections 2 and 3.1 (fourier.hip): Gaussian
// gridding on an M x M frequency grid held in centred order (grid point s
// stands for the frequency 2 pi (s - M/2) / M per dimension).
struct Fou {
    const Op *op = nullptr;          // borrowed: geometry, sizes and the solver buffers
    int32_t n = 0, M = 0, logM = 0, m_sp = 0, D = 0;   // D = 4 m_sp - 1 stencil side
    int32_t Lr = 0;                  // FFT lines per workgroup of the row passes
    int32_t dtype = 0, msize = 4, vsize = 4;
    double tau = 0.0;
    int64_t P = 0, n_tiles = 0, sp_nnz = 0, device_bytes = 0;
    int32_t *pbase = nullptr;        // [P][2]: first window cell minus (1 - m_sp), i.e. floor(xi/h) + M/2, (y, x)
    double *w1d = nullptr;           // [P][2][2 m_sp]: heat-kernel weights along y, then x
    int64_t *sp_ptr = nullptr;       // gridding B as CSR over grid points: [M*M + 1]
    int32_t *sp_pt = nullptr;        // point of each entry
    void *sp_w = nullptr;            // its weight (matrix value type)
    int32_t *sp_order = nullptr;     // grid points by descending row length
    int32_t *tile_map = nullptr;     // [(M/8)^2]: coefficient block of an 8 x 8 tile, -1 if zero
    void *coef = nullptr;            // B B^*: [n_tiles][D*D][64] (matrix value type)
    void *tw = nullptr;              // [M/2] exp(-2 pi i k / M) (vector type pairs)
    void *a1 = nullptr;              // [n] sqrt(pi/tau) exp(m^2 tau) (-1)^m / M (vector type)
    std::vector<void *> owned;
};
// out = alpha H x + lambda K^T K x + sigma x (H by path: 0 fused, 1 NUFFT);
// partial <x, out> per workgroup into part[batch][fourier_parts] when part !=
// nullptr.  grids: fourier_grid_bytes(f, batch) bytes of scratch.
template <class TM, class TV>
int launch_fourier_normal(const Fou &f, int path, double alpha, double lambda, double sigma,
                          const TV *x, TV *out, double *part, int batch, void *grids, hipStream_t s);
// x = alpha Re(F fhat), fhat [batch][P] complex.
template <class TM, class TV>
int launch_fourier_adj(const Fou &f, const TV *fhat, TV *x, double alpha, int batch, void *grids,
                       hipStream_t s);
int64_t fourier_parts(const Fou &f);
int64_t fourier_grid_bytes(const Fou &f, int batch);
// sum part[batch][count] -> dst[batch] (fixed order)
int launch_sum_partials(const double *part, int64_t count, double *dst, int batch, hipStream_t s);


}  // namespace sct
