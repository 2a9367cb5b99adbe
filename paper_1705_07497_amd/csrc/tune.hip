// Launch autotuner of an operator: times the candidate settings of
// radon_tuning on the operator's own geometry and keeps the fastest.  Tuning
// changes how the products are scheduled, never what they compute (the waves
// per item split each sum differently, so results move at the rounding level).
//
// The optional cache is a text file of lines
//   sparsect-tune <key> <fwd_waves> <adj_waves> <fwd_rhs> <adj_rhs> <fwd_layout> <fwd_lines> <adj_layout>
// (the last three may be missing: 0) keyed by GPU architecture, geometry, measured-angle set, operator kind,
// forward bundle width and batch; a later line for a key overrides an earlier
// one, and lines of other kinds are ignored.
#include "cg.hpp"

#include <cstdio>
#include <cstring>
#include <string>

namespace sct {

static int tune_key(const Op &op, int batch, std::string *key)
{
    int dev = 0;
    SCT_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    SCT_HIP(hipGetDeviceProperties(&prop, dev));
    std::string arch(prop.gcnArchName);
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    // FNV-1a over the measured angle indices
    uint64_t h = 1469598103934665603ull;
    for (int32_t k : op.meas) {
        for (int i = 0; i < 4; ++i) {
            h ^= uint64_t((uint32_t(k) >> (8 * i)) & 0xffu);
            h *= 1099511628211ull;
        }
    }
    // the bundle layout: width, angles per bundle when more than one, c when
    // compact, s when stored by symmetry
    char lay[32];
    const char *st = op.compact ? (op.sym ? "cs" : "c") : (op.sym ? "s" : "");
    if (op.bang > 1) snprintf(lay, sizeof lay, "bw%da%d%s", op.bw, op.bang, st);
    else snprintf(lay, sizeof lay, "bw%d%s", op.bw, st);
    char buf[256];
    snprintf(buf, sizeof buf, "%s|n%d|a%d|b%d|m%016llx|k%d|%s|B%d", arch.c_str(), op.n, op.n_angles,
             op.n_bins, (unsigned long long)h, op.dtype, lay, batch);
    *key = buf;
    return RADON_OK;
}

static bool lines_built(const Op &op, int lines)
{
    if (lines == 0) return true;
    for (const BandSet &b : op.bands)
        if (b.n_bands > 0 && b.lines == lines) return true;
    return false;
}

static bool tune_valid(const Op &op, const radon_tuning &t)
{
    const auto rhs_ok = [](int v) { return v == 1 || v == 4 || v == 8 || v == 16; };
    return (t.fwd_waves == 2 || t.fwd_waves == 4) &&
           (t.adj_waves == 0 || t.adj_waves == 1 || t.adj_waves == 2 || t.adj_waves == 4) &&
           rhs_ok(t.fwd_rhs) && rhs_ok(t.adj_rhs) && (t.fwd_layout == 0 || t.fwd_layout == 1) &&
           (t.adj_layout == 0 || t.adj_layout == 1) && t.reserved == 0 && lines_built(op, t.fwd_lines);
}

// Last valid entry for `key` in the cache file (false if none or no file).
static bool cache_lookup(const Op &op, const char *path, const std::string &key, radon_tuning *t)
{
    FILE *f = fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[512], k[320];
    while (fgets(line, sizeof line, f)) {
        radon_tuning c{};
        const int got = sscanf(line, "sparsect-tune %319s %d %d %d %d %d %d %d", k, &c.fwd_waves, &c.adj_waves,
                               &c.fwd_rhs, &c.adj_rhs, &c.fwd_layout, &c.fwd_lines, &c.adj_layout);
        if (got < 7) c.fwd_layout = c.fwd_lines = 0;
        if (got < 8) c.adj_layout = 0;
        if ((got == 5 || got == 7 || got == 8) && key == k && tune_valid(op, c)) {
            *t = c;
            found = true;
        }
    }
    fclose(f);
    return found;
}

static int cache_append(const char *path, const std::string &key, const radon_tuning &t)
{
    FILE *f = fopen(path, "a");
    if (!f) return set_error(RADON_EINVAL, "cannot open the tuning cache %s for writing", path);
    // one short line per write: concurrent writers append whole lines
    char line[512];
    const int len = snprintf(line, sizeof line, "sparsect-tune %s %d %d %d %d %d %d %d\n", key.c_str(),
                             t.fwd_waves, t.adj_waves, t.fwd_rhs, t.adj_rhs, t.fwd_layout, t.fwd_lines,
                             t.adj_layout);
    const bool ok = fwrite(line, 1, size_t(len), f) == size_t(len);
    fclose(f);
    if (!ok) return set_error(RADON_EINVAL, "cannot write the tuning cache %s", path);
    return RADON_OK;
}

// Forward scratch of the largest of the candidate chunkings, gather layouts
// and band heights.
static int64_t tune_part_elems(const Op &op, int batch)
{
    int64_t m = 0;
    for (int r : {1, 4, 8, 16}) {
        const int bc = r <= batch ? r : 1;
        for (int layout : {0, 1})
            for (int lines : {0, 16, 32, 64, 128}) {
                if (!lines_built(op, lines)) continue;
                const int64_t e = fwd_scratch_elems(op, bc, bc, layout, lines);
                m = e > m ? e : m;
            }
        // the adjoint's pixel-major copy of a chunk
        const int64_t a = bc >= 4 ? kPixelMajorSlack + int64_t(bc) * op.rows : 0;
        m = a > m ? a : m;
    }
    return m;
}

// Workspace of the tuner: x and its transpose, y and out for `batch` images,
// and the forward's band partials for any candidate chunking.
int64_t tune_ws_bytes(const Op &op, int batch)
{
    Carver c(nullptr);
    c.take<char>(int64_t(op.vsize) * op.nn * batch);     // x
    c.take<char>(int64_t(op.vsize) * op.nn * batch);     // x^T
    c.take<char>(int64_t(op.vsize) * op.rows * batch);   // y
    c.take<char>(int64_t(op.vsize) * op.nn * batch);     // out
    c.take<char>(int64_t(op.vsize) * tune_part_elems(op, batch));
    return c.used;
}

struct Timer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Timer()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Milliseconds per call of launch() (one untimed call first, then `reps`).
template <class F>
static int time_calls(hipStream_t s, Timer &tm, int reps, F &&launch, float *ms)
{
    SCT_TRY(launch());
    SCT_HIP(hipEventRecord(tm.e0, s));
    for (int i = 0; i < reps; ++i) SCT_TRY(launch());
    SCT_HIP(hipEventRecord(tm.e1, s));
    SCT_HIP(hipEventSynchronize(tm.e1));
    float t = 0.f;
    SCT_HIP(hipEventElapsedTime(&t, tm.e0, tm.e1));
    *ms = t / float(reps);
    return RADON_OK;
}

template <class TM, class TV>
static int tune_typed(Op &op, int batch, void *ws, hipStream_t s, radon_tuning *best)
{
    Carver c(ws);
    TV *x = c.take<TV>(op.nn * batch);
    TV *xT = c.take<TV>(op.nn * batch);
    TV *y = c.take<TV>(op.rows * batch);
    TV *out = c.take<TV>(op.nn * batch);
    const int64_t pe = tune_part_elems(op, batch);
    TV *part = pe ? c.take<TV>(pe) : nullptr;
    // a smooth positive image (the products' timing does not depend on the values)
    k_fill<TV><<<vec_blocks(op.nn * batch), kVecThreads, 0, s>>>(x, TV(0.5), op.nn * batch);
    SCT_TRY(check_launch("k_fill"));
    k_fill<TV><<<vec_blocks(op.nn * batch), kVecThreads, 0, s>>>(xT, TV(0.5), op.nn * batch);
    SCT_TRY(check_launch("k_fill"));
    Timer tm;
    SCT_HIP(hipEventCreate(&tm.e0));
    SCT_HIP(hipEventCreate(&tm.e1));
    // single-image products take tens of microseconds: 20 calls per candidate
    // keep the ranking above the run-to-run noise; fused products take
    // milliseconds, and 3 calls do
    const int reps1 = 20, reps = 3;
    best->fwd_layout = best->fwd_lines = best->adj_layout = 0;   // the search starts from the defaults
    radon_tuning cur = *best;
    auto fwd = [&](int b) {
        return [&, b]() { return launch_fwd<TM, TV>(op, x, op.need_T ? xT : nullptr, y, b, s, part); };
    };
    auto adj = [&](int b) {
        return [&, b]() { return launch_adj<TM, TV>(op, y, x, out, 1.0, 1.0, 0.0, nullptr, b, s, part); };
    };
    // one image: waves per forward bundle, then per adjoint tile
    float bt = 0.f;
    for (int w : {2, 4}) {
        op.tune = cur;
        op.tune.fwd_waves = w;
        float t = 0.f;
        SCT_TRY(time_calls(s, tm, reps1, fwd(1), &t));
        if (w == 2 || t < bt) {
            bt = t;
            best->fwd_waves = w;
        }
    }
    cur.fwd_waves = best->fwd_waves;
    for (int w : {1, 2, 4}) {
        op.tune = cur;
        op.tune.adj_waves = w;
        float t = 0.f;
        SCT_TRY(time_calls(s, tm, reps1, adj(1), &t));
        if (w == 1 || t < bt) {
            bt = t;
            best->adj_waves = w;
        }
    }
    cur.adj_waves = best->adj_waves;
    // an adjoint stored by symmetry: one workgroup per tile orbit
    // (adj_layout 1) at each wave count, against the best per-tile launch,
    // when there are at least 4 orbits per CU of the 256 (with fewer, the
    // last round of orbits leaves most CUs idle: at 512 x 512, 528 orbits,
    // the orbit kernel is faster alone but not inside the solves)
    if (op.sym_adj && op.n_orb >= 4 * 256) {
        for (int w : {1, 2, 4}) {
            op.tune = cur;
            op.tune.adj_waves = w;
            op.tune.adj_layout = 1;
            float t = 0.f;
            SCT_TRY(time_calls(s, tm, reps1, adj(1), &t));
            if (t < bt) {
                bt = t;
                best->adj_waves = w;
                best->adj_layout = 1;
            }
        }
        cur.adj_waves = best->adj_waves;
        cur.adj_layout = best->adj_layout;
    }
    // several images: how many share each matrix load, in both products
    // together (the chunkings interact through the caches), timed on the
    // normal operator's two products; then, at the best adjoint chunk, the
    // forward's gather layout and band height for each forward chunk
    if (batch > 1) {
        auto normal = [&]() {
            SCT_TRY((launch_fwd<TM, TV>(op, x, op.need_T ? xT : nullptr, y, batch, s, part)));
            return launch_adj<TM, TV>(op, y, x, out, 1.0, 1.0, 0.0, nullptr, batch, s, part);
        };
        bool first = true;
        for (int fr : {1, 4, 8, 16}) {
            if (fr > batch) continue;
            for (int ar : {1, 4, 8, 16}) {
                if (ar > batch) continue;
                op.tune = cur;
                op.tune.fwd_rhs = fr;
                op.tune.adj_rhs = ar;
                float t = 0.f;
                SCT_TRY(time_calls(s, tm, reps, normal, &t));
                if (first || t < bt) {
                    bt = t;
                    best->fwd_rhs = fr;
                    best->adj_rhs = ar;
                }
                first = false;
            }
        }
        cur.fwd_rhs = best->fwd_rhs;
        cur.adj_rhs = best->adj_rhs;
        for (int fr : {4, 8, 16}) {
            if (fr > batch) continue;
            for (int layout : {0, 1})
                for (int lines : {0, 16, 32, 64, 128}) {
                    if (!lines_built(op, lines) || (fr == cur.fwd_rhs && layout == 0 && lines == 0)) continue;
                    op.tune = cur;
                    op.tune.fwd_rhs = fr;
                    op.tune.fwd_layout = layout;
                    op.tune.fwd_lines = lines;
                    float t = 0.f;
                    SCT_TRY(time_calls(s, tm, reps, normal, &t));
                    if (t < bt) {
                        bt = t;
                        best->fwd_rhs = fr;
                        best->fwd_layout = layout;
                        best->fwd_lines = lines;
                    }
                }
        }
        cur.fwd_rhs = best->fwd_rhs;
        cur.fwd_layout = best->fwd_layout;
        cur.fwd_lines = best->fwd_lines;
        // the adjoint chunk's staging layout, for each adjoint chunk
        for (int ar : {4, 8, 16}) {
            if (ar > batch) continue;
            op.tune = cur;
            op.tune.adj_rhs = ar;
            op.tune.adj_layout = 1;
            float t = 0.f;
            SCT_TRY(time_calls(s, tm, reps, normal, &t));
            if (t < bt) {
                bt = t;
                best->adj_rhs = ar;
                best->adj_layout = 1;
            }
        }
    }
    return RADON_OK;
}

}  // namespace sct

using namespace sct;

extern "C" int radon_autotune(radon_op *p, int32_t batch, void *ws, int64_t ws_bytes,
                              const char *cache_path, int32_t flags, void *stream, int32_t *source)
{
    clear_error();
    SCT_TRY(check_op(p));
    SCT_TRY(check_batch(batch));
    if (batch > 65535) return set_error(RADON_EUNSUPPORTED, "batch %d exceeds 65535", batch);
    if (flags & ~RADON_TUNE_CACHED_ONLY) return set_error(RADON_EINVAL, "unknown flags 0x%x", flags);
    Op &op = *as_op(p);
    if (source) *source = 0;
    std::string key;
    if (cache_path) {
        SCT_TRY(tune_key(op, batch, &key));
        radon_tuning t{};
        if (cache_lookup(op, cache_path, key, &t)) {
            op.tune = t;
            if (source) *source = 1;
            return RADON_OK;
        }
    }
    if (flags & RADON_TUNE_CACHED_ONLY) return RADON_OK;
    SCT_TRY(check_ws(ws, ws_bytes, tune_ws_bytes(op, batch), "radon_autotune"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const radon_tuning before = op.tune;
    radon_tuning best = before;
    const int rc = dispatch(op, [&](auto *tm, auto *tv) {
        SCT_TYPES(tm, tv);
        return tune_typed<TM, TV>(op, batch, ws, s, &best);
    });
    if (rc != RADON_OK) {
        (void)hipStreamSynchronize(s);
        op.tune = before;
        return rc;
    }
    op.tune = best;
    if (source) *source = 2;
    if (cache_path) SCT_TRY(cache_append(cache_path, key, best));
    return RADON_OK;
}
