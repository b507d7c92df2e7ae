// Internal interfaces between the C ABI (api.hip) and the kernel files:
// the device scalar block, the workspace layout and the launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.hpp"
#include "geosstv.h"

namespace geo {

// Exact l1-ball threshold search state for one field (radix search over the
// FP32 bit patterns of |z|, see select.hip).
struct SelState {
    double radius;     // radius of the l1 ball
    double s_above;    // sum of |z| over values above the current bit range
    double tau;        // final soft-threshold level
    uint64_t c_above;  // count of those values
    uint32_t prefix;   // pattern bits fixed so far
    uint32_t done;     // tau final
    uint32_t level;    // next radix level (0, 1, 2)
    uint32_t pad;
};

constexpr int kHistBins = 2048;  // bins of radix level 0 (levels 1 and 2 use 1024)

// Per-field histogram of one radix level: counts and exact integer sums of
// the 24-bit significands (all values of a level-0 bin share one exponent).
struct Hist {
    uint32_t count[kHistBins];
    uint64_t msum[kHistBins];
};

// Scalars of the iteration kept on the device. y4 is stored lazily as
// y4 = c4 * (y4s - d4 * v / 5): the fidelity-ball step of Alg. 1 (steps
// 14-15) only rescales y4' - v/5 by max(0, 1 - eps/r), and that factor is
// applied when y4 is next read instead of in an extra pass.
struct DevScalars {
    double c4, d4;
    double r;       // ||5 y4' - v|| of the last iteration
    double rel;     // ||u+ - u|| / ||u|| of the last iteration
    double eps, tol;
    uint32_t iter;       // iterations since init
    uint32_t stop;       // stopping rule met: every kernel becomes a no-op
    uint32_t nonfinite;  // NaN/Inf seen
    uint32_t calls_iter; // iterations done in the current geo_step call
    SelState sel[2];     // 0: s (alpha), 1: t (beta)
    uint32_t fallback;   // extra threshold passes in the current call
    uint32_t pad[3];
};

// Offsets (bytes) of every region of a solver workspace.
struct Layout {
    size_t scalars, partials, hist, y4p, zs, zt;
    size_t u[2], s[2], t[2], w1[2], w2[2];  // FP32 primal, ping-pong
    size_t y1[2], y2[2], y3[2], y4[2];      // duals (FP32 or BF16), ping-pong
    size_t total;
    int dual_bytes;
    int n_part;  // number of FP64 partial-sum slots
};

// Tile of the fused primal/dual sweep.
constexpr int kTI = 8, kTJ = 64, kKC = 16, kSweepThreads = 256;
constexpr int kPointThreads = 256;

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

struct SweepGrid {
    int tj, ti, tk;  // tiles along j, i and band chunks
    int blocks() const { return tj * ti * tk; }
};
inline SweepGrid sweep_grid(int n1, int n2, int n3)
{
    return SweepGrid{ceil_div(n2, kTJ), ceil_div(n1, kTI), ceil_div(n3, kKC)};
}
inline int point_blocks(int64_t n) { return ceil_div(n, kPointThreads); }

Layout make_layout(int n1, int n2, int n3, int dual_storage);

// Pointers of one ping-pong side.
template <typename DT>
struct Side {
    float *u, *s, *t, *w1, *w2;
    DT *y1, *y2, *y3, *y4;
};

struct IterParams {
    double omega, mu_lo, mu_hi, alpha, beta;
};

// ---- launchers (kernels in sweep.hip / select.hip / ops.hip) ----
hipError_t launch_init(const Dims &d, const float *v, void *ws, const Layout &L, double eps,
                       double tol, hipStream_t st);
hipError_t launch_begin_call(void *ws, const Layout &L, double tol, hipStream_t st);
// ev (may be null): 5 events recorded at the phase boundaries
// (before sweep A, after sweep A, after the threshold search, after sweep B,
// after finalize).
hipError_t launch_iteration(const Dims &d, const float *v, void *ws, const Layout &L,
                            const IterParams &ip, hipStream_t st, hipEvent_t *ev = nullptr);
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

// Standalone projections (ops.hip).
int l2_blocks(int64_t n);
hipError_t launch_l2(const float *x, const float *c, int64_t n, double eps, float *out,
                     double *partials, double *r_dev, hipStream_t st);
hipError_t launch_prox_l12(const float *xa, const float *xb, int64_t n, float gamma, float *oa,
                           float *ob, hipStream_t st);
hipError_t launch_box(const float *x, int64_t n, float lo, float hi, float *out, hipStream_t st);

}  // namespace geo
