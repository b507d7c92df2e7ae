/*
 * geosstv.h - C ABI of the MI355X (gfx950) GeoSSTV denoising-and-destriping
 * solver: the preconditioned primal-dual splitting (P-PDS) iteration of
 * Alg. 1 in Takemoto and Ono, "Geometric Spatio-Spectral Total Variation for
 * Hyperspectral Image Denoising and Destriping", applied to problem (20)
 * (the split form of the constrained problem (15)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Cube layout. Band-sequential (BSQ): element (i, j, k) of the N1 x N2 x N3
 *   cube (i vertical pixel, j horizontal pixel, k band; Sec. II-A) is at
 *   index (k*N1 + i)*N2 + j of a float array. Multi-plane fields are planes
 *   of N floats one after another:
 *     D x, y1, y2 : [vertical, horizontal]                          2 planes
 *     L y, w1, w2 : [ud_v, ud_h, lr_v, lr_h, c_v, c_h]              6 planes
 *   where ud is the (i+1/2, j) grid, lr the (i, j+1/2) grid and c the pixel
 *   grid of Condat's interpolation operators (Sec. II-D).
 * Pointers. Every array argument is a DEVICE pointer (hipMalloc'ed or a
 *   torch CUDA tensor on the current device) owned by the caller, unless the
 *   argument says "host". The library never allocates or frees device memory:
 *   scratch lives in a caller-provided workspace sized by the matching
 *   *_workspace_size call. Outputs must not alias inputs or the workspace.
 * Streams. `stream` is a hipStream_t passed as void* (NULL = the null
 *   stream). Work is enqueued on it; calls that return scalars to the host
 *   (tau, r, the geo_result) synchronise that stream before returning.
 * Precision. Iterates are FP32, arithmetic FP32, the global quantities (the
 *   l2-ball distance, the l1-ball thresholds, the stopping norms) FP64.
 * Errors. 0 = success; positive = warning (GEO_MAXITER); negative = error.
 *   On an error nothing is guaranteed about the outputs. No call throws.
 *   Calls are thread-safe and reentrant as long as concurrent calls use
 *   distinct workspaces and outputs.
 */
#ifndef GEOSSTV_H
#define GEOSSTV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GEO_OK = 0,
    GEO_MAXITER = 1,        /* warning: iteration cap reached before tol   */
    GEO_EINVAL = -1,        /* bad dims, params, sizes or null pointers    */
    GEO_EWORKSPACE = -2,    /* workspace missing, too small or misaligned  */
    GEO_EHIP = -3,          /* a HIP runtime call failed                   */
    GEO_ENONFINITE = -4     /* NaN or Inf appeared in the iterates          */
};

/* Storage type of the dual variables y1..y4 inside the workspace. */
enum { GEO_STORE_F32 = 0, GEO_STORE_BF16 = 1 };

typedef struct {
    int32_t n1, n2, n3; /* each >= 1; N = n1*n2*n3 < 2^31. The solver
                           entry points (workspace, state, step, solve,
                           batch, geometry) also need one band to fit the
                           fused sweep's tile limit: at most 4096 tiles of
                           8 x 128 and of 16 x 64 pixels per band (up to
                           2048 x 2048 pixels); larger bands give
                           GEO_EINVAL. The operator and projection entry
                           points take any dims above.                     */
} geo_dims;

/* Parameters of problem (15) and of the loop of Alg. 1. The step sizes are
 * not parameters: they are the constants printed after eq. (24)
 * (u 1/13, w1 1/4, w2 1/4, s 1, t 1/3, y1..y4 1/5). */
typedef struct {
    double eps;          /* radius of the fidelity ball (18), >= 0          */
    double alpha;        /* radius of the sparse-noise l1 ball (16), >= 0   */
    double beta;         /* radius of the stripe-noise l1 ball (17), >= 0   */
    double mu_lo, mu_hi; /* box (19), mu_lo < mu_hi                         */
    double omega;        /* GeoSSTV balance of eq. (13), >= 0               */
    int32_t max_iter;    /* iteration cap, >= 1 (geo_solve)                 */
    double tol;          /* stop after the first iteration with
                            ||u+ - u||_2 / ||u||_2 < tol (eq. (28)), not
                            counting the first iteration after
                            geo_state_init (from zero duals it changes u
                            only by the box projection); tol <= 0 runs
                            exactly max_iter iterations                    */
    int32_t dual_storage;/* GEO_STORE_F32 or GEO_STORE_BF16                 */
    int32_t check_every; /* iterations between host checks of the stopping
                            flag (0 = 32); the count returned is exact
                            whatever this is, since the device stops
                            iterating on its own once the rule is met      */
    int32_t band_chunk;  /* bands each tile of the fused sweep marches
                            through (0 = chosen per cube: the depth in 8..32
                            whose tiles the device's persistent blocks finish
                            first, see geo_sweep_geometry; values below 8
                            count as 8; raised when a cube would have more
                            than 4096 tiles). A performance knob only:
                            results do not depend on it beyond FP64
                            summation order.                              */
    int32_t regularizer; /* GEO_REG_GEOSSTV (0, the method of the paper) or
                            one of the regularizers it compares against
                            (Sec. IV-A), in the same constrained problem
                            (15) and solved by the same P-PDS (eq. (7)):
                              GEO_REG_SSTV    ||D D_s u||_1
                              GEO_REG_HSSTV1  ||(D D_s u, omega D u)||_1
                              GEO_REG_HSSTV2  sum over voxels of the l2
                                              norm of the 4 entries of
                                              (D D_s u, omega D u) there
                            with step sizes from eq. (8) and the operator
                            norm bounds ||D D_s||^2 <= 32, ||omega D||^2
                            <= 8 omega^2, ||D_v||^2 <= 4: u 1/33 (SSTV) or
                            1/(33 + 8 omega^2), s 1, t 1/5, duals 1/3. The
                            variants take GEO_STORE_F32 only, geo_workspace_
                            size, geo_state_init/get/set, geo_step,
                            geo_step_timed (it times the dual kernel) and
                            geo_solve (not the batched or profiled entry
                            points: GEO_EINVAL), and any dims with
                            N < 2^31. Their state: u, s, t, y1 (2 planes
                            [D_v D_s u, D_h D_s u] for SSTV, 4 for HSSTV
                            with [omega D_v u, omega D_h u] after them), y3
                            (D_v t) and y4 (u + s + t); w1, w2 and y2 do
                            not exist (GEO_EINVAL). They use the same
                            exact l1 threshold search (windows, histogram
                            passes of a missed window in the same slot),
                            so every geo_result field has its meaning.    */
} geo_params;

enum { GEO_REG_GEOSSTV = 0, GEO_REG_SSTV = 1, GEO_REG_HSSTV1 = 2, GEO_REG_HSSTV2 = 3 };

typedef struct {
    int32_t iters;       /* iterations performed by this call               */
    int32_t converged;   /* 1 if the stopping rule was met                  */
    double rel_change;   /* ||u+ - u|| / ||u|| of the last iteration         */
    double r;            /* ||y4'/gamma - v||_2 of the last iteration        */
    double tau_s, tau_t; /* soft-threshold levels of the last l1 projections
                            (0 inside the ball, +inf for a zero radius)     */
    int32_t total_iters; /* iterations since geo_state_init                  */
    int32_t fallback_passes; /* l1 thresholds found by the full search (the
                                predicted window missed) during the call   */
    int32_t cand_s, cand_t;  /* values inside the predicted windows in the
                                last iteration (diagnostic)                */
    int32_t slots;       /* launch slots the call issued (one iteration of
                            every working cube each; a missed window is
                            resolved inside its slot)                       */
    int32_t status;      /* this cube's own status: GEO_OK, GEO_MAXITER or
                            GEO_ENONFINITE (a batch returns the worst)      */
} geo_result;

/* Workspace of a solver state for one cube (bytes, 256-byte aligned base
 * required). Errors: GEO_EINVAL for bad dims/params. */
int geo_workspace_size(geo_dims dims, const geo_params *p, size_t *bytes);

/* Set the state of Alg. 1 to its initial point: u = v, every other
 * variable zero (the paper leaves the initial point open; this is the
 * reading used). v: N floats. */
int geo_state_init(geo_dims dims, const geo_params *p, const float *v,
                   void *ws, size_t ws_bytes, void *stream);

/* Run up to n_iter iterations of Alg. 1 (steps 1-15) on the state in ws,
 * stopping early by the rule of eq. (28) when p->tol > 0. v must be the cube
 * the state was initialised with. Blocking: fills *out (may be NULL).
 * Returns GEO_OK, GEO_MAXITER (tol > 0 and not met) or an error. */
int geo_step(geo_dims dims, const geo_params *p, const float *v,
             void *ws, size_t ws_bytes, int32_t n_iter, void *stream,
             geo_result *out);

/* geo_step with HIP events recorded at the phase boundaries of every
 * iteration on `stream` (instrumentation for benchmarks; the events add a
 * few microseconds per iteration). phase_ms (host, GEO_NPHASE doubles)
 * receives the summed GPU time of each phase over the call:
 *   0 sweep A  (steps 1, 4, 5, 11, 12 and the u' part of 14 fused, plus the
 *              inputs of the threshold search)
 *   1 the exact soft-threshold search of the two l1-ball projections
 *   2 sweep B  (steps 2, 3, 13, the rest of 14, the l2-ball factor of step
 *              15 and the stopping rule) */
#define GEO_NPHASE 3
int geo_step_profiled(geo_dims dims, const geo_params *p, const float *v,
                      void *ws, size_t ws_bytes, int32_t n_iter, void *stream,
                      geo_result *out, double *phase_ms);

/* geo_step with two HIP events around the fused sweep (for the comparison
 * regularizers: their dual kernel) of the 8th, 16th, ... iteration slot of
 * the call (the first slot follows a host synchronisation and starts from
 * an idle device), or of every slot in calls of fewer than 8, on `stream`:
 * the kernel's launch time for a roofline. An event pair idles the GPU for
 * a few microseconds, so sampling keeps that cost out of 7 of 8 iterations.
 * *sweep_a_ms (host) receives the GPU time of that kernel summed over the
 * call, estimated as the mean of the sampled launches times the number of
 * slots (iterations done, for the regularizers). */
int geo_step_timed(geo_dims dims, const geo_params *p, const float *v,
                   void *ws, size_t ws_bytes, int32_t n_iter, void *stream,
                   geo_result *out, double *sweep_a_ms);

/* geo_state_init + geo_step(max_iter) + copy of u, s, t (N floats each). */
int geo_solve(geo_dims dims, const geo_params *p, const float *v,
              float *u, float *s, float *t, void *ws, size_t ws_bytes,
              void *stream, geo_result *out);

/* Batched iterations: n_cubes independent solver states (cubes of any sizes,
 * each initialised by geo_state_init in its own workspace) advanced together,
 * one launch sequence per iteration for all of them: the fused sweep runs
 * persistently over the concatenated tiles of the cubes still working, the
 * threshold search and the finalisation take one block per cube and field.
 * Each cube does n_iter iterations of Alg. 1 or stops earlier by its own
 * rule (eq. (28), its p[c].tol); a cube that is done idles while the others
 * go on, so every cube's iterates are exactly those geo_step would give it
 * alone.
 *   dims, p, v, ws, ws_bytes, out: HOST arrays of n_cubes entries (v[c] and
 *       ws[c] are device pointers); every p[c].dual_storage must be equal.
 *   table: device buffer of geo_batch_table_size bytes (256-byte aligned)
 *       for the launch table; it may be reused by later calls.
 *   use_graph != 0: one iteration's launch sequence is captured into a HIP
 *       graph and replayed (fewer launches on the host). The instantiated
 *       graph is kept (up to 16 per process) and replayed by later calls on
 *       the same device with the same table address, storage and cube
 *       sizes; the table's contents are uploaded by every call.
 * Blocking; returns GEO_ENONFINITE if any cube saw NaN/Inf, else GEO_MAXITER
 * if any cube with tol > 0 did not meet its rule, else GEO_OK. 1 <= n_cubes
 * <= 64. */
int geo_batch_table_size(int32_t n_cubes, size_t *bytes);
int geo_batch_step(int32_t n_cubes, const geo_dims *dims, const geo_params *p,
                   const float *const *v, void *const *ws, const size_t *ws_bytes,
                   void *table, size_t table_bytes, int32_t n_iter, int32_t use_graph,
                   void *stream, geo_result *out);

/* Launch geometry of the fused sweep (steps 1, 4, 5, 11, 12 of Alg. 1 and
 * the inputs of steps 2 and 3), for callers that model load balance, such
 * as a band-chunk autotuner. Host-side only: no GPU work.
 *   dual_storage: GEO_STORE_F32 or GEO_STORE_BF16 (as in geo_params). A
 *       tile is 8 x 128 pixels, or 16 x 64 when the cube's width fills a
 *       64-wide tile grid more than 3% better (FP32 duals only).
 *   requested: bands per tile asked for; the library uses at least 8 and
 *       doubles it until the cube has at most 4096 tiles. 0 = the default:
 *       the depth kc in 8..32 that minimises ceil(tiles / blocks) x
 *       (min(kc, n3) + 2), ties to the deeper one.
 *   blocks: persistent blocks the default is chosen for (geo_sweep_blocks
 *       on the device that will run the cube); read only when requested = 0.
 *   used_chunk: the bands per tile the library will use.
 *   tiles: tiles of this cube at that chunk (pixel tiles x band chunks).
 *   tile_rows, tile_cols: pixel shape of a tile (n1 rows x n2 columns).
 * Errors: GEO_EINVAL for bad dims or storage type, requested < 0,
 * requested = 0 with blocks < 1, or a NULL output. */
int geo_sweep_geometry(geo_dims dims, int32_t dual_storage, int32_t requested, int32_t blocks,
                       int32_t *used_chunk, int32_t *tiles, int32_t *tile_rows,
                       int32_t *tile_cols);

/* Tile capacity of a solver workspace for these dims and storage: the
 * most tiles any band chunk that geo_sweep_geometry can report (for every
 * request and block count) gives the cube. The per-tile regions of the
 * workspace (partial sums, window statistics, candidate counts) hold that
 * many tiles. Host-only; no device needed.
 * Errors: GEO_EINVAL for bad dims, storage type or a NULL output. */
int geo_workspace_tiles(geo_dims dims, int32_t dual_storage, int32_t *max_tiles);

/* Persistent blocks of the fused sweep on the current device: a launch
 * runs min(blocks, tiles of all its cubes) blocks, and each block takes
 * tiles in turn. dual_storage: GEO_STORE_F32 or GEO_STORE_BF16.
 * Errors: GEO_EINVAL for a bad storage type or NULL output; GEO_EHIP
 * without a usable device. */
int geo_sweep_blocks(int32_t dual_storage, int32_t *blocks);

/* State variables, for parity tests, checkpointing and resume. */
enum {
    GEO_VAR_U = 0, GEO_VAR_S, GEO_VAR_T, GEO_VAR_W1, GEO_VAR_W2,
    GEO_VAR_Y1, GEO_VAR_Y2, GEO_VAR_Y3, GEO_VAR_Y4
};

/* Copy a state variable out of / into the workspace in FP32 (planes as
 * above: 1 for u, s, t, y3, y4; 6 for w1, w2; 2 for y1, y2). p gives the
 * storage type of the workspace. Loading any state is allowed, including
 * entries the operators never read. v may be NULL (the workspace keeps y4
 * in a scaled residual form that does not need it). Asynchronous. */
int geo_state_get(geo_dims dims, const geo_params *p, const void *ws, size_t ws_bytes,
                  int32_t var, const float *v, float *out, void *stream);
int geo_state_set(geo_dims dims, const geo_params *p, void *ws, size_t ws_bytes,
                  int32_t var, const float *v, const float *in, void *stream);

/* Linear operators of problem (20) (Sec. II-A differences with the Neumann
 * boundary; Condat's interpolation operators of Sec. II-D in the reading
 * where dual edge fields live on interior edges only). Asynchronous.
 *   op               forward            planes in -> out
 *   GEO_OP_DV        D_v (along i)       1 -> 1
 *   GEO_OP_DH        D_h (along j)       1 -> 1
 *   GEO_OP_DS        D_s (along k)       1 -> 1
 *   GEO_OP_D         (D_v; D_h)          1 -> 2
 *   GEO_OP_DDS       D D_s               1 -> 2
 *   GEO_OP_L_UD      L_ud                2 -> 2
 *   GEO_OP_L_LR      L_lr                2 -> 2
 *   GEO_OP_L_C       L_c                 2 -> 2
 *   GEO_OP_L         (L_ud; L_lr; L_c)   2 -> 6
 *   GEO_OP_K         stacked operator of (20): (u,s,t,w1,w2) 15 -> 6 (y1..y4)
 * adjoint != 0 applies the transpose (planes out -> in). */
enum {
    GEO_OP_DV = 0, GEO_OP_DH, GEO_OP_DS, GEO_OP_D, GEO_OP_DDS,
    GEO_OP_L_UD, GEO_OP_L_LR, GEO_OP_L_C, GEO_OP_L, GEO_OP_K
};
int geo_apply_op(int32_t op, int32_t adjoint, geo_dims dims, const float *in,
                 float *out, void *stream);

/* Projection onto {z : ||z||_1 <= radius} (constraints (16), (17); exact:
 * soft threshold at the tau with sum max(|x|-tau, 0) = radius, found by a
 * deterministic radix search over the FP32 bit patterns with exact integer
 * bin sums). x, out: n floats (may alias). *tau (host) receives the level
 * (0 inside the ball, +inf for radius 0). Blocking. */
int geo_project_l1_workspace_size(int64_t n, size_t *bytes);
int geo_project_l1(const float *x, int64_t n, double radius, float *out,
                   double *tau, void *ws, size_t ws_bytes, void *stream);

/* geo_project_l1 for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same results, with the scratch in a fixed 32 KiB device
 * array of the library (one per GPU, kept until the process ends) instead of
 * a workspace. Allocates nothing, copies nothing to the host, does not
 * synchronise. tau_dev: DEVICE pointer to one double receiving the level (0
 * inside the ball, +inf for radius 0), or NULL. n <= 2^31 - 1, else
 * GEO_EINVAL. Every call on a GPU uses that GPU's one scratch array: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller. */
int geo_project_l1_noalloc(const float *x, int64_t n, double radius, float *out,
                           double *tau_dev, void *stream);

/* Projection onto the ball of radius eps around center, eq. (23). *r (host)
 * receives ||x - center||_2 (FP64). Blocking. */
int geo_project_l2_workspace_size(int64_t n, size_t *bytes);
int geo_project_l2(const float *x, const float *center, int64_t n, double eps,
                   float *out, double *r, void *ws, size_t ws_bytes, void *stream);

/* Prox of gamma ||.||_{1,2}, eq. (24), on groups (xa[q], xb[q]). */
int geo_prox_l12(const float *xa, const float *xb, int64_t n, double gamma,
                 float *oa, float *ob, void *stream);

/* Box projection, eq. (21). */
int geo_project_box(const float *x, int64_t n, double lo, double hi, float *out,
                    void *stream);

const char *geo_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* GEOSSTV_H */
