// Internal interfaces between the C ABI (api.hip) and the kernel files:
// the device scalar block, the workspace layout and the launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.hpp"
#include "geosstv.h"

namespace geo {

// Exact l1-ball threshold search state for one field. In steady state the
// level tau moves little between iterations: sweep A collects the values of
// |z| inside a window [win_lo, win_hi] predicted from the last two levels
// (candidates) plus the count and sum of the values above it, and one block
// finishes the search exactly over the candidates. When the window misses,
// a radix search over the FP32 bit patterns of the whole field runs instead,
// in the same launch slot (fallback.hip, radix.hpp).
struct SelState {
    double radius;     // radius of the l1 ball
    double s_above;    // radix search: sum of |z| above the current bit range
    double tau;        // soft-threshold level of this iteration
    double tau_prev;   // level of the previous iteration (window prediction)
    double tau_prev2;  // and of the one before
    double tau_prev3;  // and of the one before that
    uint64_t c_above;  // radix search: count of those values
    uint32_t prefix;   // radix search: pattern bits fixed so far
    uint32_t done;     // tau final for this iteration
    uint32_t level;    // next radix level (0, 1, 2)
    uint32_t full;     // 1 when the radix search over the full field runs
    float win_lo, win_hi;  // window used by the next sweep A
    uint32_t win_on;       // window valid
    uint32_t cand_count;   // candidates in the window (search bookkeeping)
    double dens;           // values of |z| per unit near tau in the last
                           // iteration (sizes the next window)
};

constexpr int kHistBins = 2048;  // bins of radix level 0 (levels 1 and 2 use 1024)

// Per-field histogram of one radix level: counts and exact integer sums of
// the 24-bit significands (all values of a level-0 bin share one exponent).
struct Hist {
    uint32_t count[kHistBins];
    uint64_t msum[kHistBins];
};

// Outcome of one radix level of a field whose window missed, written by the
// histogram pass of that level (fallback.hip) and read by the next pass,
// sweep B and the finalize of the same launch slot.
struct FbRec {
    double tau;      // the threshold, when the level ended the search
    double s_above;  // sum and count of the values above the chosen bin
    double c_above;
    double dens;     // values per unit of |z| in tau's level-0 bin (level 0)
    uint32_t prefix; // bits fixed so far (the chosen bins)
    uint32_t done;   // the level ended the search
};

// The threshold of a field that missed its window, from the records of this
// slot's passes: the first level that ended the search.
__host__ __device__ inline const FbRec &fb_final(const FbRec *rec, int f)
{
    return rec[0 * 2 + f].done ? rec[0 * 2 + f] : (rec[1 * 2 + f].done ? rec[1 * 2 + f] : rec[2 * 2 + f]);
}

// Scalars of the iteration kept on the device. y4 is stored as the residual
// q = 5 y4' - v with y4 = a4 * q: the fidelity-ball step of Alg. 1 (steps
// 14-15, eq. (23) through the conjugate prox) only rescales y4' - v/5 = q/5
// by c4 = max(0, 1 - eps/r), r = ||q||, and that factor is applied when y4
// is next read instead of in an extra pass. The residual form keeps y4 free
// of the cancellation y4' - v/5 (y4' is close to v/5), also in BF16.
struct DevScalars {
    double c4, a4;  // last factor of step 15; y4 = a4 * stored
    double r;       // ||5 y4' - v|| of the last iteration
    double rel;     // ||u+ - u|| / ||u|| of the last iteration
    double eps, tol;
    uint32_t iter;       // iterations since init
    uint32_t stop;       // stopping rule met: every kernel becomes a no-op
    uint32_t nonfinite;  // NaN/Inf seen
    uint32_t calls_iter; // iterations done in the current geo_step call
    SelState sel[2];     // 0: s (alpha), 1: t (beta)
    uint32_t fallback;   // full radix searches in the current call
    uint32_t call_limit; // iterations this call may do: the cube idles after them
    uint32_t zstore;     // sweep A of this iteration stores z_s and z_t
    uint32_t calm;       // iterations in a row whose windows all held tau
    double gy4;          // step of y4: after an iteration y4 = gy4 c4 q
};

// Iterations in which a threshold window is likely to miss store the inputs
// of the two l1 projections as sweep A computes them (8 bytes per voxel), so
// that the histogram passes of a missed window read 4 bytes per voxel and
// field instead of evaluating them again from the state (16 bytes per
// voxel). Likely: the first kZStoreIters iterations after the initial point
// or a state load (tau moves fast while the duals build up), and until
// kZStoreCalm iterations in a row have held their windows after a miss.
constexpr uint32_t kZStoreIters = 16;
constexpr uint32_t kZStoreCalm = 3;

// A cube whose stopping rule holds, or that has done the iterations of the
// current call, turns every kernel of a launch slot into a no-op.
__device__ __forceinline__ bool idle(const DevScalars *sc)
{
    return sc->stop || sc->calls_iter >= sc->call_limit;
}

// Offsets (bytes) of every region of a solver workspace.
struct Layout {
    size_t scalars, partials, hist, rec, y4p, winpart, cand, ccount, zbuf, table;
    size_t u[2], s[2], t[2], w1[2], w2[2];  // FP32 primal, ping-pong
    size_t y1[2], y2[2], y3[2], y4[2];      // duals (FP32 or BF16), ping-pong
    size_t total;
    int dual_bytes;
    int n_part;     // FP64 partial-sum slots: 2 per tile, then sweep B blocks
    int max_tiles;  // most sweep A tiles of any band chunk the library may use
    int64_t cap;    // candidate capacity per field
};

// Tile of the fused primal/dual sweep: TI x TJ pixels (one per thread of a
// 1024-thread workgroup), marching through a chunk of kc bands (kc chosen
// per cube at run time). Two shapes, chosen per cube by its width:
//   shape 0, 8 x 128: each band row of a tile is one 512-byte run per array;
//     it streamed 2.5% faster than 16 x 64 in a probe of the same 22-read,
//     18-write access pattern;
//   shape 1, 16 x 64: for widths that leave much of a 128-column tile
//     outside the cube (N2 = 160: 37.5% of the lanes of two 128-wide tiles,
//     17% of three 64-wide ones). Idle lanes cost time, since the sweep's
//     rate is set by its loads in flight.
constexpr int kTileShapes = 2;
constexpr int kShapeTI[kTileShapes] = {8, 16}, kShapeTJ[kTileShapes] = {128, 64};
constexpr int kSweepThreads = 1024;
constexpr int kDefaultKC = 32;       // deepest default chunk (the rule below picks 8..32)
constexpr int kMinKC = 8;
constexpr int kMaxTiles = 4096;      // tiles of one cube (slices of its search)
constexpr int kMaxBatch = 64;        // cubes of one batched launch
constexpr int kPointThreads = 256;
constexpr int kSweepBBlocks = 2048;  // grid-stride blocks of sweep B per cube
constexpr int kSweepBRows = 2;       // rows of a sweep B strip
constexpr int kTimedEvery = 8;  // geo_step_timed: events around every 8th sweep A

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Tile shape of a cube: 16 x 64 when its share of tile points inside the
// cube beats that of 8 x 128 by more than 3% (the streaming advantage of the
// wider tile), else 8 x 128. With BF16 duals always 8 x 128 (the 16 x 64
// sweep spills registers in that form). A function of the cube's size and
// storage only, so a cube runs the same tiles alone and in a batch.
inline double tile_fill(int n1, int n2, int shape)
{
    const int ti = kShapeTI[shape], tj = kShapeTJ[shape];
    return ((double)n1 / (ti * ceil_div(n1, ti))) * ((double)n2 / (tj * ceil_div(n2, tj)));
}
inline int tile_shape(int n1, int n2, int dual_bytes)
{
    return dual_bytes == 4 && tile_fill(n1, n2, 1) > 1.03 * tile_fill(n1, n2, 0) ? 1 : 0;
}
struct SweepGrid {
    int tj, ti, tk, kc;  // tiles along j, i, band chunks; bands per chunk
    int shape;           // tile shape (kShapeTI/kShapeTJ)
    __host__ __device__ int blocks() const { return tj * ti * tk; }
};
inline SweepGrid sweep_grid(int n1, int n2, int n3, int kc, int shape)
{
    return SweepGrid{ceil_div(n2, kShapeTJ[shape]), ceil_div(n1, kShapeTI[shape]), ceil_div(n3, kc), kc,
                     shape};
}
// Fixed work of one tile (its halo band, the pipeline fill, its partial
// sums) in band-equivalents, for the load-balance rule below.
constexpr double kTileFixedBands = 2.0;
// Default depth for a cube: the chunk in [kMinKC, kDefaultKC] whose tiles,
// taken in turn by `blocks` persistent blocks, finish first. A round of
// tiles costs the deepest tile's bands plus the fixed work; ties keep the
// deeper chunk (fewer tiles). A cube with few tiles gets shallower chunks,
// so that more blocks work on it, and a tile count just past a multiple of
// the blocks is avoided. blocks <= 0: kDefaultKC.
inline int default_chunk(int n1, int n2, int n3, int blocks, int shape)
{
    if (blocks <= 0) return kDefaultKC;
    int best = kDefaultKC;
    double best_cost = 0.0;
    for (int kc = kDefaultKC; kc >= kMinKC; --kc) {
        const SweepGrid g = sweep_grid(n1, n2, n3, kc, shape);
        const int T = g.blocks();
        if (T > kMaxTiles) break;  // shallower chunks only add tiles
        const int G = blocks < T ? blocks : T;
        const double cost = (double)ceil_div(T, G) * ((kc < n3 ? kc : n3) + kTileFixedBands);
        if (kc == kDefaultKC || cost < best_cost - 1e-9) {
            best = kc;
            best_cost = cost;
        }
    }
    return best;
}
// Pixel tiles of one band.
inline int tiles_per_band(int n1, int n2, int shape)
{
    return ceil_div(n2, kShapeTJ[shape]) * ceil_div(n1, kShapeTI[shape]);
}
// A cube the solver takes: one band of it fits the tile limit in either
// shape, so some band chunk always does.
inline bool solver_dims_fit(int n1, int n2)
{
    for (int q = 0; q < kTileShapes; ++q)
        if ((int64_t)ceil_div(n2, kShapeTJ[q]) * ceil_div(n1, kShapeTI[q]) > kMaxTiles) return false;
    return true;
}
// Bands per tile actually used: the request (0 = the default above for
// `blocks` persistent blocks), at least kMinKC, raised until the cube has at
// most kMaxTiles tiles (always reached for a cube that solver_dims_fit
// takes: at kc >= n3 a cube has one band chunk).
inline int band_chunk(int n1, int n2, int n3, int requested, int blocks, int shape)
{
    int kc = requested > 0 ? requested : default_chunk(n1, n2, n3, blocks, shape);
    if (kc < kMinKC) kc = kMinKC;
    while (kc < n3 && sweep_grid(n1, n2, n3, kc, shape).blocks() > kMaxTiles) kc *= 2;
    return kc;
}
inline int point_blocks(int64_t n) { return ceil_div(n, kPointThreads); }
inline int sweep_b_blocks(int64_t n)
{
    int b = point_blocks(n);
    return b < kSweepBBlocks ? b : kSweepBBlocks;
}
// Most tiles band_chunk can give the cube, for any request and block count
// and either shape: the tile count falls as the chunk deepens, so it is the
// count at the shallowest chunk >= kMinKC within the limit. The per-tile
// regions of the workspace (partials, window statistics, candidate counts)
// are sized by it.
inline int max_tiles(int n1, int n2, int n3)
{
    int m = 0;
    for (int q = 0; q < kTileShapes; ++q)
        for (int kc = kMinKC;; ++kc) {
            const int t = sweep_grid(n1, n2, n3, kc, q).blocks();
            if (t <= kMaxTiles || kc >= n3) {
                m = t > m ? t : m;
                break;
            }
        }
    return m;
}

Layout make_layout(int n1, int n2, int n3, int dual_storage);

// Pointers of one ping-pong side. Inside the workspace the two components
// of each dual edge field and of each l_{1,2} group of w sit together:
//   y1, y2 : N pairs (vertical, horizontal)
//   w1, w2 : 3 planes of N pairs, one plane per grid (ud, lr, c)
// (the ABI's state accessors convert to and from separate planes).
template <typename DT>
struct Side {
    using P = typename PairOf<DT>::type;
    float *u, *s, *t;
    float2 *w1, *w2;  // 6 floats per voxel each: see w_udlr, w_c
    P *y1, *y2;
    DT *y3, *y4;
};

// Layout of w1 and w2 (6N floats each): the ud and lr pairs of a voxel side
// by side, [ud_v, ud_h, lr_v, lr_h] (N float4), then the c pairs (N float2),
// so that sweep A moves one field of a voxel in a 16-byte and an 8-byte
// access.
__host__ __device__ inline float4 *w_udlr(float2 *w) { return reinterpret_cast<float4 *>(w); }
__host__ __device__ inline const float4 *w_udlr(const float2 *w) { return reinterpret_cast<const float4 *>(w); }
__host__ __device__ inline float2 *w_c(float2 *w, int64_t n) { return w + 2 * n; }
__host__ __device__ inline const float2 *w_c(const float2 *w, int64_t n) { return w + 2 * n; }
// pair g (0 ud, 1 lr, 2 c) of voxel q
__host__ __device__ inline float2 *w_pair(float2 *w, int64_t n, int g, int64_t q)
{
    return g < 2 ? w + 2 * q + g : w + 2 * n + q;
}

// Everything the iteration kernels need about one cube. A launch covers a
// table of these in device memory (one entry for a single cube, up to
// kMaxBatch for a batch): sweep A walks the concatenated tile list of the
// cubes still working, the search takes one block per (cube, field), sweep B
// a block range per cube and the finalize one block per cube. Stopped cubes
// are skipped.
struct CubeCommon {
    Dims d;
    const float *v;
    DevScalars *sc;
    double *part;       // [2 * ntiles] tile partials (du2, u2), then sweep B blocks
    double *winpart;    // [2][ntiles][3] count above, sum above, sum of |z|
    Hist *hist;         // [3 levels][2 fields] histograms of the full threshold search
    FbRec *rec;         // [3 levels][2 fields] their outcomes
    float *cand;        // [2][ntiles][capt] candidate slices of the tiles
    uint32_t *ccount;   // [2][ntiles] candidates appended by each tile
    float *zbuf;        // [2][N] z_s, z_t of an iteration that stores them
    int capt;           // candidate capacity of one tile slice
    int ntiles;
    SweepGrid g;
    int tile0;          // first tile of this cube in the launch's full tile list
    int b0, nb;         // sweep B blocks of this cube: first, count
    float thr1;         // omega * step of w1
    float zt_step;      // step size of t in z_t (the histogram passes evaluate z_t)
    float mu_lo, mu_hi;
    // sweep B's inputs by side parity (s, t, y3, y4, the y4 intermediate)
    // and their sizes, for the cache prefetch that runs beside the search
    const void *bin[2][5];
    size_t bin_bytes[5];
};
template <typename DT>
struct CubeArgs {
    CubeCommon c;
    Side<DT> side[2];
    DT *y4p;            // 5 y4 + u' - v: step 14 before s', t'
};

// Read-only view of a launch table through the constant address space: its
// loads are invariant, so the compiler may issue them again where needed
// instead of keeping every field live in registers (as for kernel
// arguments). Structs are read field by field.
template <typename T>
using const4 = const __attribute__((address_space(4))) T;

template <typename DT>
__device__ __forceinline__ Side<DT> load_side(const4<Side<DT>> &s)
{
    Side<DT> o;
    o.u = s.u;
    o.s = s.s;
    o.t = s.t;
    o.w1 = s.w1;
    o.w2 = s.w2;
    o.y1 = s.y1;
    o.y2 = s.y2;
    o.y3 = s.y3;
    o.y4 = s.y4;
    return o;
}
__device__ __forceinline__ Dims load_dims(const4<Dims> &d)
{
    Dims o;
    o.n1 = d.n1;
    o.n2 = d.n2;
    o.n3 = d.n3;
    o.plane = d.plane;
    return o;
}

// Shape of one launch slot over a table of cubes.
struct LaunchShape {
    int ncubes;
    int total_tiles;  // sweep A tiles over all cubes
    int grid_a;       // persistent sweep A blocks
    int total_b;      // sweep B blocks over all cubes
    int shape_tiles[kTileShapes];  // sweep A tiles of the cubes of each tile shape
    int shape_grid[kTileShapes];   // persistent blocks of the sweep A launch of each shape
    int fb_grid;      // blocks of each fallback histogram pass
    int b_kinds;      // sweep B forms present: 1 one or two columns per thread, 2 four
};

// Columns per sweep B thread for a row length: four when it is a multiple of
// 4 (16-byte FP32 and 8-byte BF16 accesses), else two when it is even, else
// one. dual_bytes: storage of the duals (the same rule for both).
__host__ __device__ inline int sweep_b_cpt(int n2, int dual_bytes)
{
    (void)dual_bytes;
    return (n2 & 1) ? 1 : ((n2 & 3) == 0 ? 4 : 2);
}

// Host image of one cube's table entry (FP32 or BF16 duals: same size).
struct CubeEntry {
    unsigned char bytes[sizeof(CubeArgs<float>)];
};
static_assert(sizeof(CubeArgs<float>) == sizeof(CubeArgs<bf16>), "one table entry size");

// Launch-wide words of a table, in the 512 bytes after its entries (the
// table upload zeroes them). Word 0: set by the window search when some
// threshold of the slot missed its window, cleared by the finalize; the
// histogram passes leave at once when it is 0. Words 64 + c (their own
// cache lines, touched only by atomics of system scope): blocks of the
// running histogram pass done with cube c.
constexpr size_t kTableFlagBytes = 512;
constexpr int kFbCounterWord = 64;
__host__ __device__ inline size_t table_flags_offset(int ncubes)
{
    return ((size_t)ncubes * sizeof(CubeEntry) + 255) & ~(size_t)255;
}
__host__ __device__ inline uint32_t *slot_flags(const void *table, int ncubes)
{
    return (uint32_t *)((char *)table + table_flags_offset(ncubes));
}
__host__ __device__ inline size_t table_bytes(int ncubes) { return table_flags_offset(ncubes) + kTableFlagBytes; }

// ---- launchers (kernels in sweep.hip / select.hip / ops.hip) ----
hipError_t launch_init(const Dims &d, const float *v, void *ws, const Layout &L, double eps,
                       double tol, double alpha, double beta, hipStream_t st);
hipError_t launch_begin_call(void *ws, const Layout &L, double tol, double alpha, double beta,
                             int call_limit, hipStream_t st);
// Fill e for the cube (d, v, ws) with band chunk kc; tile0/b0 place it in
// the launch; returns its tile and sweep B block counts.
void cube_entry(CubeEntry *e, const Dims &d, const float *v, void *ws, const Layout &L, double omega,
                double mu_lo, double mu_hi, int kc, int tile0, int b0, int *ntiles, int *nb);
int sweep_a_grid(int dual_bytes, int total_tiles);
// One launch slot over the table (device copy of the entries). ev (may be
// null): nev = 4 events recorded at the phase boundaries (before sweep A,
// after sweep A, after the threshold search, after sweep B and the
// finalize), or nev = 2 around sweep A only.
hipError_t launch_slot(const void *table, int dual_bytes, const LaunchShape &sh, hipStream_t st,
                       hipEvent_t *ev = nullptr, int nev = 4);
// out != null: copy the variable out (FP32); otherwise load it from in.
hipError_t launch_state_io(const Dims &d, void *ws, const Layout &L, int var, const float *v,
                           float *out, const float *in, hipStream_t st);
hipError_t launch_apply_op(int op, int adjoint, const Dims &d, const float *in, float *out,
                           hipStream_t st);
int op_planes(int op, int adj, int *pin, int *pout);

// Exact l1-ball threshold search (select.hip). stop may be null.
hipError_t select_begin(SelState *sel, int nfields, double r0, double r1, Hist *hist,
                        const uint32_t *stop, hipStream_t st);
hipError_t select_run(const float *z0, const float *z1, int nfields, int64_t n, SelState *sel,
                      Hist *hist, const uint32_t *stop, hipStream_t st);
hipError_t launch_l1_threshold(const float *x, int64_t n, double radius, SelState *sel,
                               Hist *hist, hipStream_t st);
hipError_t launch_soft(const float *x, int64_t n, const SelState *sel, float *out, hipStream_t st);
// The solver's per-iteration search over a table of cubes (entries of
// `stride` bytes, CubeCommon first): one block per (cube, field).
// Extra blocks of the same launch stream sweep B's inputs through the
// memory-side cache meanwhile (prefetch_blocks, 0 = none).
hipError_t launch_select_window(const void *table, int stride, int ncubes, int prefetch_blocks,
                                hipStream_t st);

// The histogram pass of radix level `level` (0..2) for the thresholds whose
// window missed in this slot (fallback.hip); a no-op when none did.
int fallback_grid();
hipError_t launch_fallback(const void *table, int dual_bytes, const LaunchShape &sh, int level,
                           hipStream_t st);

// The comparison regularizers (variants.hip): problem (15) with SSTV or
// HSSTV in place of GeoSSTV, with the same device scalars, window search,
// histogram passes and finalize as the main solver.
int var_planes(int regularizer);
size_t var_workspace_bytes(int n1, int n2, int n3, int regularizer);
hipError_t var_state_init(const Dims &d, const geo_params *p, const float *v, void *ws,
                          hipStream_t st);
// n_iter iterations or fewer once the rule of eq. (28) holds; blocking;
// fills *out with the device scalars. dual_ms (may be null): GPU time of the
// dual kernel over the call, from events around a sample of launches.
hipError_t var_step(const Dims &d, const geo_params *p, const float *v, void *ws, int n_iter,
                    hipStream_t st, DevScalars *out, int *slots, double *dual_ms = nullptr);
// out != null: copy the variable out; otherwise load it from in.
hipError_t var_state_io(const Dims &d, const geo_params *p, void *ws, int var, float *out,
                        const float *in, hipStream_t st);

// The finalize of a launch slot over a table of ncubes entries of `stride`
// bytes (sweep.hip), and the scalar reset after a state load.
hipError_t launch_finalize(const void *table, int stride, int ncubes, hipStream_t st);
hipError_t launch_state_loaded(DevScalars *sc, int var, hipStream_t st);

// GEO_OK for hipSuccess, else GEO_EHIP with the error kept for
// geo_strerror (api.hip).
int geo_hip_status(hipError_t e);

// Standalone projections (ops.hip).
int l2_blocks(int64_t n);
hipError_t launch_l2(const float *x, const float *c, int64_t n, double eps, float *out,
                     double *partials, double *r_dev, hipStream_t st);
hipError_t launch_prox_l12(const float *xa, const float *xb, int64_t n, float gamma, float *oa,
                           float *ob, hipStream_t st);
hipError_t launch_box(const float *x, int64_t n, float lo, float hi, float *out, hipStream_t st);

}  // namespace geo
