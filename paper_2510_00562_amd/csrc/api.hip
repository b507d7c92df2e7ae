// extern "C" entry points declared in include/geosstv.h: argument checks,
// workspace carving and launch sequencing. No device memory is allocated
// here; every buffer is the caller's.
#include <math.h>
#include <string.h>

#include <memory>
#include <type_traits>
#include <mutex>
#include <vector>

#include "solver.hpp"

namespace geo {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout make_layout(int n1, int n2, int n3, int dual_storage)
{
    Layout L;
    memset(&L, 0, sizeof L);
    const size_t N = (size_t)n1 * n2 * n3;
    const size_t f4 = N * sizeof(float);
    const int db = dual_storage == GEO_STORE_BF16 ? 2 : 4;
    const size_t fd = N * db;
    L.dual_bytes = db;
    L.max_tiles = max_tiles(n1, n2, n3);
    L.n_part = 2 * L.max_tiles + sweep_b_blocks((int64_t)N);
    L.cap = (int64_t)N / 16 > 65536 ? (int64_t)N / 16 : 65536;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.scalars = take(sizeof(DevScalars));
    L.partials = take(sizeof(double) * (size_t)L.n_part);
    L.hist = take(6 * sizeof(Hist));  // 3 radix levels x 2 fields
    L.rec = take(6 * sizeof(FbRec));
    L.y4p = take(fd);
    L.winpart = take(sizeof(double) * 2 * 3 * (size_t)L.max_tiles);
    L.cand = take(sizeof(float) * 2 * (size_t)L.cap);
    L.ccount = take(sizeof(uint32_t) * 2 * (size_t)L.max_tiles);
    L.zbuf = take(2 * f4);
    L.table = take(table_bytes(1));
    for (int p = 0; p < 2; ++p) {
        L.u[p] = take(f4);
        L.s[p] = take(f4);
        L.t[p] = take(f4);
        L.w1[p] = take(6 * f4);
        L.w2[p] = take(6 * f4);
        L.y1[p] = take(2 * fd);
        L.y2[p] = take(2 * fd);
        L.y3[p] = take(fd);
        L.y4[p] = take(fd);
    }
    L.total = o;
    return L;
}

}  // namespace geo

using namespace geo;

namespace {

thread_local hipError_t g_last_hip = hipSuccess;

// Instantiated graphs of one launch slot, reused across calls. A slot's
// kernels take only the table's address and the launch shape (the table's
// contents are uploaded before every call and read by the kernels), so a
// graph captured for the same device, table address, storage and shape is
// the same graph. A request loop that keeps its batch for several rounds
// then pays the capture and instantiation once. At most kGraphCache graphs
// are kept (the oldest leaves first); a graph is destroyed when it has left
// the cache and no call still replays it.
struct GraphKey {
    int device;
    int dual_bytes;
    const void *table;
    LaunchShape sh;
};
using GraphRef = std::shared_ptr<std::remove_pointer<hipGraphExec_t>::type>;
constexpr size_t kGraphCache = 16;
std::mutex g_graph_mu;
// never destroyed: the graphs still cached at exit are left to the runtime's
// own teardown rather than destroyed after it
std::vector<std::pair<GraphKey, GraphRef>> &graph_cache()
{
    static auto *v = new std::vector<std::pair<GraphKey, GraphRef>>();
    return *v;
}

GraphRef cached_graph(const GraphKey &k)
{
    std::lock_guard<std::mutex> lock(g_graph_mu);
    for (auto &e : graph_cache())
        if (memcmp(&e.first, &k, sizeof k) == 0) return e.second;
    return nullptr;
}

GraphRef keep_graph(const GraphKey &k, hipGraphExec_t g)
{
    GraphRef ref(g, [](hipGraphExec_t x) { (void)hipGraphExecDestroy(x); });
    std::lock_guard<std::mutex> lock(g_graph_mu);
    auto &c = graph_cache();
    if (c.size() >= kGraphCache) c.erase(c.begin());
    c.emplace_back(k, ref);
    return ref;
}

int hip_status(hipError_t e)
{
    if (e == hipSuccess) return GEO_OK;
    g_last_hip = e;
    return GEO_EHIP;
}

bool dims_ok(geo_dims d)
{
    if (d.n1 < 1 || d.n2 < 1 || d.n3 < 1) return false;
    const int64_t N = (int64_t)d.n1 * d.n2 * d.n3;
    return N < ((int64_t)1 << 31);
}

// Cubes the solver entry points take: one band within the tile limit.
bool solver_dims_ok(geo_dims d) { return dims_ok(d) && solver_dims_fit(d.n1, d.n2); }

bool finite_nonneg(double x) { return isfinite(x) && x >= 0.0; }

bool params_ok(const geo_params *p)
{
    if (!p) return false;
    if (!finite_nonneg(p->eps) || !finite_nonneg(p->alpha) || !finite_nonneg(p->beta)) return false;
    if (!finite_nonneg(p->omega)) return false;
    if (!isfinite(p->mu_lo) || !isfinite(p->mu_hi) || !(p->mu_lo < p->mu_hi)) return false;
    if (isnan(p->tol)) return false;
    if (p->dual_storage != GEO_STORE_F32 && p->dual_storage != GEO_STORE_BF16) return false;
    if (p->check_every < 0) return false;
    if (p->band_chunk < 0) return false;
    if (p->regularizer < GEO_REG_GEOSSTV || p->regularizer > GEO_REG_HSSTV2) return false;
    if (p->regularizer != GEO_REG_GEOSSTV && p->dual_storage != GEO_STORE_F32) return false;
    return true;
}

bool is_variant(const geo_params *p) { return p && p->regularizer != GEO_REG_GEOSSTV; }

Dims to_dims(geo_dims d)
{
    Dims x;
    x.n1 = d.n1;
    x.n2 = d.n2;
    x.n3 = d.n3;
    x.plane = (int64_t)d.n1 * d.n2 * d.n3;
    return x;
}

int check_ws(geo_dims d, const geo_params *p, const void *ws, size_t ws_bytes, Layout *L)
{
    *L = make_layout(d.n1, d.n2, d.n3, p ? p->dual_storage : GEO_STORE_F32);
    if (!ws || ((uintptr_t)ws & 255u) || ws_bytes < L->total) return GEO_EWORKSPACE;
    return GEO_OK;
}

hipStream_t S(void *stream) { return (hipStream_t)stream; }

// The comparison regularizers (variants.hip): any dims with N < 2^31.
int check_var_ws(geo_dims d, const geo_params *p, const void *ws, size_t ws_bytes)
{
    if (!ws || ((uintptr_t)ws & 255u) || ws_bytes < var_workspace_bytes(d.n1, d.n2, d.n3, p->regularizer))
        return GEO_EWORKSPACE;
    return GEO_OK;
}

int var_step_impl(geo_dims dims, const geo_params *p, const float *v, void *ws, size_t ws_bytes,
                  int32_t n_iter, hipStream_t st, geo_result *out, double *dual_ms = nullptr)
{
    int rc = check_var_ws(dims, p, ws, ws_bytes);
    if (rc) return rc;
    DevScalars x;
    int slots = 0;
    rc = hip_status(var_step(to_dims(dims), p, v, ws, n_iter, st, &x, &slots, dual_ms));
    if (rc) return rc;
    const int own = x.nonfinite ? GEO_ENONFINITE : (p->tol > 0.0 && !x.stop ? GEO_MAXITER : GEO_OK);
    if (out) {
        memset(out, 0, sizeof *out);
        out->iters = (int32_t)x.calls_iter;
        out->converged = (p->tol > 0.0 && x.stop && !x.nonfinite) ? 1 : 0;
        out->rel_change = x.rel;
        out->r = x.r;
        out->tau_s = x.sel[0].tau;
        out->tau_t = x.sel[1].tau;
        out->total_iters = (int32_t)x.iter;
        out->fallback_passes = (int32_t)x.fallback;
        out->cand_s = (int32_t)x.sel[0].cand_count;
        out->cand_t = (int32_t)x.sel[1].cand_count;
        out->slots = (int32_t)slots;
        out->status = own;
    }
    return own;
}

int read_scalars(const void *ws, const Layout &L, DevScalars *out, hipStream_t st)
{
    hipError_t e = hipMemcpyAsync(out, (const char *)ws + L.scalars, sizeof(DevScalars),
                                  hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_status(e);
    return hip_status(hipStreamSynchronize(st));
}

}  // namespace

namespace geo {
// For entry points in other files: the status of a HIP call, keeping the
// error for geo_strerror.
int geo_hip_status(hipError_t e) { return hip_status(e); }
}  // namespace geo

extern "C" {

const char *geo_strerror(int status)
{
    switch (status) {
    case GEO_OK: return "success";
    case GEO_MAXITER: return "iteration cap reached before the stopping rule held";
    case GEO_EINVAL: return "invalid argument (dims, parameters, sizes or null pointer)";
    case GEO_EWORKSPACE: return "workspace missing, misaligned (256 B) or too small";
    case GEO_EHIP: return hipGetErrorString(g_last_hip);
    case GEO_ENONFINITE: return "NaN or Inf appeared in the iterates";
    default: return "unknown status";
    }
}

int geo_workspace_size(geo_dims dims, const geo_params *p, size_t *bytes)
{
    if (is_variant(p)) {
        if (!dims_ok(dims) || !bytes || !params_ok(p)) return GEO_EINVAL;
        *bytes = var_workspace_bytes(dims.n1, dims.n2, dims.n3, p->regularizer);
        return GEO_OK;
    }
    if (!solver_dims_ok(dims) || !bytes) return GEO_EINVAL;
    if (p && (p->dual_storage != GEO_STORE_F32 && p->dual_storage != GEO_STORE_BF16))
        return GEO_EINVAL;
    *bytes = make_layout(dims.n1, dims.n2, dims.n3, p ? p->dual_storage : GEO_STORE_F32).total;
    return GEO_OK;
}

int geo_state_init(geo_dims dims, const geo_params *p, const float *v, void *ws, size_t ws_bytes,
                   void *stream)
{
    if (is_variant(p)) {
        if (!dims_ok(dims) || !params_ok(p) || !v) return GEO_EINVAL;
        const int rc = check_var_ws(dims, p, ws, ws_bytes);
        return rc ? rc : hip_status(var_state_init(to_dims(dims), p, v, ws, S(stream)));
    }
    if (!solver_dims_ok(dims) || !params_ok(p) || !v) return GEO_EINVAL;
    Layout L;
    int rc = check_ws(dims, p, ws, ws_bytes, &L);
    if (rc) return rc;
    return hip_status(launch_init(to_dims(dims), v, ws, L, p->eps, p->tol, p->alpha, p->beta,
                                  S(stream)));
}

// One solver call over n cubes (n = 1: the single-cube entry points). The
// launch table (host image `ent`, device copy at `table`) is written once;
// each launch slot (sweep A, search, the three histogram passes of a missed
// window, sweep B, finalize) completes one iteration of every busy cube.
// With a tolerance the host reads the stopping flags every check_every
// slots; the device idles a cube once it has met its rule or done n_iter
// iterations.
// phase_ms (may be null): nph = GEO_NPHASE phase times (4 events in every
// slot), or nph = 1 for sweep A alone: 2 events around it in every
// kTimedEvery-th slot, from the kTimedEvery-th on (the first slot of a call
// follows a host synchronisation and starts from an idle device), the
// sampled times scaled to all slots (an event pair costs a few
// microseconds of idle time between the launches it brackets, which
// sampling keeps out of most iterations).
static int run_cubes(int n, const geo_dims *dims, const geo_params *p, const float *const *v,
                     void *const *ws, const size_t *ws_bytes, void *table, size_t table_bytes_given,
                     int32_t n_iter, int use_graph, hipStream_t st, geo_result *out,
                     double *phase_ms, int nph = GEO_NPHASE)
{
    if (n < 1 || n > kMaxBatch || !dims || !p || !v || !ws || !ws_bytes || n_iter < 0)
        return GEO_EINVAL;
    std::vector<Layout> L(n);
    for (int c = 0; c < n; ++c) {
        if (!solver_dims_ok(dims[c]) || !params_ok(&p[c]) || !v[c] || is_variant(&p[c])) return GEO_EINVAL;
        if (p[c].dual_storage != p[0].dual_storage) return GEO_EINVAL;
        int rc = check_ws(dims[c], &p[c], ws[c], ws_bytes[c], &L[c]);
        if (rc) return rc;
    }
    if (!table || ((uintptr_t)table & 255u) || table_bytes_given < table_bytes(n)) return GEO_EWORKSPACE;
    std::vector<CubeEntry> ent(n);
    LaunchShape sh{};
    sh.ncubes = n;
    for (int c = 0; c < n; ++c) {
        int nt = 0, nb = 0;
        cube_entry(&ent[c], to_dims(dims[c]), v[c], ws[c], L[c], p[c].omega, p[c].mu_lo, p[c].mu_hi,
                   p[c].band_chunk, sh.total_tiles, sh.total_b, &nt, &nb);
        // the workspace's per-tile regions hold every chunk band_chunk gives
        // (make_layout); this only guards that invariant
        if (nt > L[c].max_tiles) return GEO_EWORKSPACE;
        sh.total_tiles += nt;
        sh.total_b += nb;
        sh.shape_tiles[tile_shape(dims[c].n1, dims[c].n2, L[c].dual_bytes)] += nt;
        sh.b_kinds |= sweep_b_cpt(dims[c].n2, L[c].dual_bytes) == 4 ? 2 : 1;
    }
    sh.grid_a = sweep_a_grid(L[0].dual_bytes, sh.total_tiles);
    sh.fb_grid = fallback_grid();
    for (int q = 0; q < kTileShapes; ++q)
        sh.shape_grid[q] = sh.shape_tiles[q] > 0 ? sweep_a_grid(L[0].dual_bytes, sh.shape_tiles[q]) : 0;
    // the entries, then the launch flags zeroed
    std::vector<unsigned char> img(table_bytes(n), 0);
    memcpy(img.data(), ent.data(), (size_t)n * sizeof(CubeEntry));
    int rc = hip_status(hipMemcpyAsync(table, img.data(), img.size(), hipMemcpyHostToDevice, st));
    for (int c = 0; c < n && !rc; ++c)
        rc = hip_status(launch_begin_call(ws[c], L[c], p[c].tol, p[c].alpha, p[c].beta, n_iter, st));
    if (rc) return rc;
    const int nev = nph == 1 ? 2 : 4;
    // calls shorter than the sampling period time every slot
    const int ev_every = nph == 1 && n_iter >= kTimedEvery ? kTimedEvery : 1;
    long slots = 0, sampled = 0;
    if (phase_ms)
        for (int q = 0; q < nph; ++q) phase_ms[q] = 0.0;
    bool any_tol = false;
    for (int c = 0; c < n; ++c) any_tol = any_tol || p[c].tol > 0.0;
    const int every = p[0].check_every > 0 ? p[0].check_every : 32;

    hipGraphExec_t gexec = nullptr;
    GraphRef gref;  // keeps the graph alive while this call replays it
    hipGraph_t graph = nullptr;
    GraphKey gkey;
    memset(&gkey, 0, sizeof gkey);  // compared bytewise, padding included
    if (use_graph && !phase_ms) {
        gkey.dual_bytes = L[0].dual_bytes;
        gkey.table = table;
        gkey.sh = sh;
        rc = hip_status(hipGetDevice(&gkey.device));
        if (!rc) gref = cached_graph(gkey);
        gexec = gref.get();
    }
    const bool new_graph = use_graph && !phase_ms && !rc && !gexec;
    if (new_graph) {
        // one slot captured on a private stream (capture needs a non-null
        // stream), replayed on the caller's
        hipStream_t cs = nullptr;
        rc = hip_status(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        if (!rc) rc = hip_status(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        if (!rc) {
            hipError_t le = launch_slot(table, L[0].dual_bytes, sh, cs, nullptr);
            hipError_t ee = hipStreamEndCapture(cs, &graph);
            rc = hip_status(le != hipSuccess ? le : ee);
        }
        if (!rc) rc = hip_status(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
        if (cs) (void)hipStreamDestroy(cs);
        if (graph) (void)hipGraphDestroy(graph);  // the instantiated graph is independent of it
        graph = nullptr;
        if (!rc) gref = keep_graph(gkey, gexec);
        else if (gexec) {
            (void)hipGraphExecDestroy(gexec);
            gexec = nullptr;
        }
    }

    std::vector<DevScalars> sc(n);
    std::vector<hipEvent_t> ev;
    int behind = n_iter;  // slots still needed by the furthest-behind busy cube
    while (!rc) {
        const int batch = (any_tol && behind > every) ? every : behind;
        if (phase_ms) {
            const size_t need = (size_t)nev * (batch / ev_every + 1);
            while (ev.size() < need && !rc) {
                hipEvent_t e;
                rc = hip_status(hipEventCreate(&e));
                if (!rc) ev.push_back(e);
            }
        }
        int nsamp = 0;  // slots of this batch with events, in order
        for (int q = 0; q < batch && !rc; ++q) {
            const bool timed = phase_ms && (slots + q) % ev_every == ev_every - 1;
            if (gexec)
                rc = hip_status(hipGraphLaunch(gexec, st));
            else
                rc = hip_status(launch_slot(table, L[0].dual_bytes, sh, st,
                                            timed ? &ev[(size_t)nev * nsamp] : nullptr, nev));
            nsamp += timed ? 1 : 0;
        }
        slots += batch;
        sampled += nsamp;
        for (int c = 0; c < n && !rc; ++c)
            rc = hip_status(hipMemcpyAsync(&sc[c], (const char *)ws[c] + L[c].scalars, sizeof(DevScalars),
                                           hipMemcpyDeviceToHost, st));
        if (!rc) rc = hip_status(hipStreamSynchronize(st));
        if (!rc && phase_ms)
            for (int q = 0; q < nsamp && !rc; ++q)
                for (int ph = 0; ph < nph && !rc; ++ph) {
                    float ms = 0.f;
                    rc = hip_status(hipEventElapsedTime(&ms, ev[(size_t)nev * q + ph],
                                                        ev[(size_t)nev * q + ph + 1]));
                    phase_ms[ph] += ms;
                }
        behind = 0;
        for (int c = 0; c < n; ++c) {
            const int left = sc[c].stop ? 0 : n_iter - (int)sc[c].calls_iter;
            if (left > behind) behind = left;
        }
        if (batch == 0 || behind <= 0) break;
    }
    if (phase_ms && sampled > 0 && sampled < slots)
        for (int q = 0; q < nph; ++q) phase_ms[q] *= (double)slots / (double)sampled;
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (graph) (void)hipGraphDestroy(graph);  // a capture that failed before instantiation
    if (rc) return rc;
    int status = GEO_OK;
    for (int c = 0; c < n; ++c) {
        const DevScalars &x = sc[c];
        if (out) {
            geo_result &o = out[c];
            o.iters = (int32_t)x.calls_iter;
            o.converged = (p[c].tol > 0.0 && x.stop && !x.nonfinite) ? 1 : 0;
            o.rel_change = x.rel;
            o.r = x.r;
            o.tau_s = x.sel[0].tau;
            o.tau_t = x.sel[1].tau;
            o.total_iters = (int32_t)x.iter;
            o.fallback_passes = (int32_t)x.fallback;
            o.cand_s = (int32_t)x.sel[0].cand_count;
            o.cand_t = (int32_t)x.sel[1].cand_count;
            o.slots = (int32_t)slots;
        }
        const int own = x.nonfinite ? GEO_ENONFINITE : (p[c].tol > 0.0 && !x.stop ? GEO_MAXITER : GEO_OK);
        if (out) out[c].status = own;
        if (own == GEO_ENONFINITE) status = GEO_ENONFINITE;
        else if (status == GEO_OK && own == GEO_MAXITER) status = GEO_MAXITER;
    }
    return status;
}

static int step_impl(geo_dims dims, const geo_params *p, const float *v, void *ws, size_t ws_bytes,
                     int32_t n_iter, void *stream, geo_result *out, double *phase_ms,
                     int nph = GEO_NPHASE)
{
    if (is_variant(p)) {
        // geo_step_timed (nph = 1) times the dual kernel; no phase profile
        if (!dims_ok(dims) || !params_ok(p) || !v || n_iter < 0 || (phase_ms && nph != 1))
            return GEO_EINVAL;
        return var_step_impl(dims, p, v, ws, ws_bytes, n_iter, S(stream), out, phase_ms);
    }
    if (!solver_dims_ok(dims) || !params_ok(p) || !v || n_iter < 0) return GEO_EINVAL;
    Layout L;
    int rc = check_ws(dims, p, ws, ws_bytes, &L);
    if (rc) return rc;
    void *table = (char *)ws + L.table;
    return run_cubes(1, &dims, p, &v, &ws, &ws_bytes, table, table_bytes(1), n_iter, 0, S(stream),
                     out, phase_ms, nph);
}

int geo_step(geo_dims dims, const geo_params *p, const float *v, void *ws, size_t ws_bytes,
             int32_t n_iter, void *stream, geo_result *out)
{
    return step_impl(dims, p, v, ws, ws_bytes, n_iter, stream, out, nullptr);
}

int geo_step_profiled(geo_dims dims, const geo_params *p, const float *v, void *ws, size_t ws_bytes,
                      int32_t n_iter, void *stream, geo_result *out, double *phase_ms)
{
    if (!phase_ms) return GEO_EINVAL;
    return step_impl(dims, p, v, ws, ws_bytes, n_iter, stream, out, phase_ms);
}

int geo_step_timed(geo_dims dims, const geo_params *p, const float *v, void *ws, size_t ws_bytes,
                   int32_t n_iter, void *stream, geo_result *out, double *sweep_a_ms)
{
    if (!sweep_a_ms) return GEO_EINVAL;
    return step_impl(dims, p, v, ws, ws_bytes, n_iter, stream, out, sweep_a_ms, 1);
}

int geo_solve(geo_dims dims, const geo_params *p, const float *v, float *u, float *s, float *t,
              void *ws, size_t ws_bytes, void *stream, geo_result *out)
{
    if (!params_ok(p) || p->max_iter < 1 || !u || !s || !t) return GEO_EINVAL;
    int rc = geo_state_init(dims, p, v, ws, ws_bytes, stream);
    if (rc) return rc;
    const int step_rc = geo_step(dims, p, v, ws, ws_bytes, p->max_iter, stream, out);
    if (step_rc < 0) return step_rc;
    if (is_variant(p)) {
        const Dims d = to_dims(dims);
        const hipStream_t st = S(stream);
        rc = hip_status(var_state_io(d, p, ws, GEO_VAR_U, u, nullptr, st));
        if (!rc) rc = hip_status(var_state_io(d, p, ws, GEO_VAR_S, s, nullptr, st));
        if (!rc) rc = hip_status(var_state_io(d, p, ws, GEO_VAR_T, t, nullptr, st));
        if (!rc) rc = hip_status(hipStreamSynchronize(st));
        return rc ? rc : step_rc;
    }
    Layout L = make_layout(dims.n1, dims.n2, dims.n3, p->dual_storage);
    const Dims d = to_dims(dims);
    const hipStream_t st = S(stream);
    rc = hip_status(launch_state_io(d, ws, L, GEO_VAR_U, v, u, nullptr, st));
    if (!rc) rc = hip_status(launch_state_io(d, ws, L, GEO_VAR_S, v, s, nullptr, st));
    if (!rc) rc = hip_status(launch_state_io(d, ws, L, GEO_VAR_T, v, t, nullptr, st));
    if (!rc) rc = hip_status(hipStreamSynchronize(st));
    return rc ? rc : step_rc;
}

int geo_batch_table_size(int32_t n_cubes, size_t *bytes)
{
    if (n_cubes < 1 || n_cubes > kMaxBatch || !bytes) return GEO_EINVAL;
    *bytes = table_bytes(n_cubes);
    return GEO_OK;
}

int geo_sweep_geometry(geo_dims dims, int32_t dual_storage, int32_t requested, int32_t blocks,
                       int32_t *used_chunk, int32_t *tiles, int32_t *tile_rows, int32_t *tile_cols)
{
    if (!solver_dims_ok(dims) || (dual_storage != GEO_STORE_F32 && dual_storage != GEO_STORE_BF16) ||
        requested < 0 || (requested == 0 && blocks < 1) || !used_chunk || !tiles || !tile_rows ||
        !tile_cols)
        return GEO_EINVAL;
    const int shape = tile_shape(dims.n1, dims.n2, dual_storage == GEO_STORE_BF16 ? 2 : 4);
    const int kc = band_chunk(dims.n1, dims.n2, dims.n3, requested, blocks, shape);
    *used_chunk = kc;
    *tiles = sweep_grid(dims.n1, dims.n2, dims.n3, kc, shape).blocks();
    *tile_rows = kShapeTI[shape];
    *tile_cols = kShapeTJ[shape];
    return GEO_OK;
}

int geo_workspace_tiles(geo_dims dims, int32_t dual_storage, int32_t *max_tiles_out)
{
    if (!solver_dims_ok(dims) || (dual_storage != GEO_STORE_F32 && dual_storage != GEO_STORE_BF16) ||
        !max_tiles_out)
        return GEO_EINVAL;
    *max_tiles_out = make_layout(dims.n1, dims.n2, dims.n3, dual_storage).max_tiles;
    return GEO_OK;
}

int geo_sweep_blocks(int32_t dual_storage, int32_t *blocks)
{
    if ((dual_storage != GEO_STORE_F32 && dual_storage != GEO_STORE_BF16) || !blocks) return GEO_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GEO_EHIP;
    // the persistent grid of a launch with at least this many tiles
    *blocks = sweep_a_grid(dual_storage == GEO_STORE_BF16 ? 2 : 4, 1 << 30);
    return GEO_OK;
}

int geo_batch_step(int32_t n_cubes, const geo_dims *dims, const geo_params *p,
                   const float *const *v, void *const *ws, const size_t *ws_bytes, void *table,
                   size_t table_bytes, int32_t n_iter, int32_t use_graph, void *stream,
                   geo_result *out)
{
    return run_cubes(n_cubes, dims, p, v, ws, ws_bytes, table, table_bytes, n_iter, use_graph ? 1 : 0,
                     S(stream), out, nullptr);
}

static int state_io(geo_dims dims, const void *ws, size_t ws_bytes, int32_t var, const float *v,
                    float *out, const float *in, int dual_storage, void *stream)
{
    if (!solver_dims_ok(dims) || var < GEO_VAR_U || var > GEO_VAR_Y4) return GEO_EINVAL;
    if (dual_storage != GEO_STORE_F32 && dual_storage != GEO_STORE_BF16) return GEO_EINVAL;
    if ((out == nullptr) == (in == nullptr)) return GEO_EINVAL;
    geo_params p;
    memset(&p, 0, sizeof p);
    p.dual_storage = dual_storage;
    Layout L;
    int rc = check_ws(dims, &p, ws, ws_bytes, &L);
    if (rc) return rc;
    return hip_status(launch_state_io(to_dims(dims), (void *)ws, L, var, v, out, in, S(stream)));
}

static int var_state_call(geo_dims dims, const geo_params *p, const void *ws, size_t ws_bytes,
                          int32_t var, float *out, const float *in, void *stream)
{
    if (!dims_ok(dims) || !params_ok(p)) return GEO_EINVAL;
    if (var != GEO_VAR_U && var != GEO_VAR_S && var != GEO_VAR_T && var != GEO_VAR_Y1 &&
        var != GEO_VAR_Y3 && var != GEO_VAR_Y4)
        return GEO_EINVAL;
    const int rc = check_var_ws(dims, p, ws, ws_bytes);
    return rc ? rc : hip_status(var_state_io(to_dims(dims), p, (void *)ws, var, out, in, S(stream)));
}

int geo_state_get(geo_dims dims, const geo_params *p, const void *ws, size_t ws_bytes, int32_t var,
                  const float *v, float *out, void *stream)
{
    if (!out || !p) return GEO_EINVAL;
    if (is_variant(p)) return var_state_call(dims, p, ws, ws_bytes, var, out, nullptr, stream);
    return state_io(dims, ws, ws_bytes, var, v, out, nullptr, p->dual_storage, stream);
}

int geo_state_set(geo_dims dims, const geo_params *p, void *ws, size_t ws_bytes, int32_t var,
                  const float *v, const float *in, void *stream)
{
    if (!in || !p) return GEO_EINVAL;
    if (is_variant(p)) return var_state_call(dims, p, ws, ws_bytes, var, nullptr, in, stream);
    return state_io(dims, ws, ws_bytes, var, v, nullptr, in, p->dual_storage, stream);
}

int geo_apply_op(int32_t op, int32_t adjoint, geo_dims dims, const float *in, float *out,
                 void *stream)
{
    int pin, pout;
    if (!dims_ok(dims) || !in || !out || op_planes(op, adjoint ? 1 : 0, &pin, &pout)) return GEO_EINVAL;
    return hip_status(launch_apply_op(op, adjoint ? 1 : 0, to_dims(dims), in, out, S(stream)));
}

int geo_project_l1_workspace_size(int64_t n, size_t *bytes)
{
    if (n < 0 || !bytes) return GEO_EINVAL;
    *bytes = align256(sizeof(SelState)) + sizeof(Hist);
    return GEO_OK;
}

int geo_project_l1(const float *x, int64_t n, double radius, float *out, double *tau, void *ws,
                   size_t ws_bytes, void *stream)
{
    if (n < 0 || !isfinite(radius) || radius < 0.0 || (n > 0 && (!x || !out))) return GEO_EINVAL;
    size_t need;
    geo_project_l1_workspace_size(n, &need);
    if (!ws || ((uintptr_t)ws & 255u) || ws_bytes < need) return GEO_EWORKSPACE;
    const hipStream_t st = S(stream);
    SelState *sel = (SelState *)ws;
    Hist *hist = (Hist *)((char *)ws + align256(sizeof(SelState)));
    int rc = hip_status(launch_l1_threshold(x, n, radius, sel, hist, st));
    if (!rc && n > 0) rc = hip_status(launch_soft(x, n, sel, out, st));
    SelState h;
    if (!rc) rc = hip_status(hipMemcpyAsync(&h, sel, sizeof h, hipMemcpyDeviceToHost, st));
    if (!rc) rc = hip_status(hipStreamSynchronize(st));
    if (!rc && tau) *tau = h.tau;
    return rc;
}

int geo_project_l2_workspace_size(int64_t n, size_t *bytes)
{
    if (n < 0 || !bytes) return GEO_EINVAL;
    *bytes = align256(sizeof(double) * (size_t)l2_blocks(n > 0 ? n : 1)) + 256;
    return GEO_OK;
}

int geo_project_l2(const float *x, const float *center, int64_t n, double eps, float *out, double *r,
                   void *ws, size_t ws_bytes, void *stream)
{
    if (n < 1 || !x || !center || !out || !isfinite(eps) || eps < 0.0) return GEO_EINVAL;
    size_t need;
    geo_project_l2_workspace_size(n, &need);
    if (!ws || ((uintptr_t)ws & 255u) || ws_bytes < need) return GEO_EWORKSPACE;
    const hipStream_t st = S(stream);
    double *part = (double *)ws;
    double *rd = (double *)((char *)ws + align256(sizeof(double) * (size_t)l2_blocks(n)));
    int rc = hip_status(launch_l2(x, center, n, eps, out, part, rd, st));
    double h = 0.0;
    if (!rc) rc = hip_status(hipMemcpyAsync(&h, rd, sizeof h, hipMemcpyDeviceToHost, st));
    if (!rc) rc = hip_status(hipStreamSynchronize(st));
    if (!rc && r) *r = h;
    return rc;
}

int geo_prox_l12(const float *xa, const float *xb, int64_t n, double gamma, float *oa, float *ob,
                 void *stream)
{
    if (n < 0 || !isfinite(gamma) || gamma < 0.0) return GEO_EINVAL;
    if (n == 0) return GEO_OK;
    if (!xa || !xb || !oa || !ob) return GEO_EINVAL;
    return hip_status(launch_prox_l12(xa, xb, n, (float)gamma, oa, ob, S(stream)));
}

int geo_project_box(const float *x, int64_t n, double lo, double hi, float *out, void *stream)
{
    if (n < 0 || !isfinite(lo) || !isfinite(hi) || !(lo < hi)) return GEO_EINVAL;
    if (n == 0) return GEO_OK;
    if (!x || !out) return GEO_EINVAL;
    return hip_status(launch_box(x, n, (float)lo, (float)hi, out, S(stream)));
}

}  // extern "C"
