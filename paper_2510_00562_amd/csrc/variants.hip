// Problem (15) with the GeoSSTV term replaced by one of the regularizers the
// paper compares against (Sec. IV-A), solved by the same P-PDS (eq. (7)):
//   SSTV:   ||D D_s u||_1
//   HSSTV1: ||(D D_s u, omega D u)||_1
//   HSSTV2: sum over voxels of the l2 norm of (D D_s u, omega D u) there
// Primal blocks (u, s, t), dual blocks (y1 for A u, y3 for D_v t, y4 for
// u + s + t); step sizes from eq. (8) with the operator-norm bounds
// ||D D_s||^2 <= 32, ||omega D||^2 <= 8 omega^2, ||D_v||^2 <= 4:
//   u 1/(||A||^2 + 1), s 1, t 1/5, y 1/3.
//
// One iteration, on the caller's stream:
//   primal kernel: u+ = P_box(u - g_u (A^T y1 + y4)) into the other u buffer,
//                  the inputs z_s = s - y4 and z_t = t - g_t (D_v^T y3 + y4)
//                  of the two l1-ball projections, FP64 partials of the
//                  stopping rule;
//   threshold search: the exact radix search of the standalone l1
//                  projection over z_s and z_t;
//   dual kernel:   s+, t+ (soft thresholds), the extrapolations x' = 2 x+ - x,
//                  y1 += g_y A u' and the conjugate prox of the regularizer
//                  (a clip to [-1, 1], or each 4-entry group scaled into the
//                  unit l2 ball), y3 += g_y D_v t', the y4 residual and FP64
//                  partials of its norm;
//   finalize:      the fidelity-ball factor (y4 - g_y P_B(y4/g_y) =
//                  c g_y (y4/g_y - v), c = max(0, 1 - eps/r), applied when y4
//                  is next read), the relative change, the stopping rule.
// A plain path on purpose: streaming kernels with grid-stride loops, the
// stencils read through the caches, no tile fusion.
#include <math.h>
#include <string.h>

#include <vector>

#include "solver.hpp"

namespace geo {

namespace {

constexpr int VT = 256;               // threads of the streaming kernels
// Their grid: one voxel per thread up to this many blocks (2M voxels),
// grid-stride beyond; one FP64 partial per block and sum. 8192 blocks of 4
// wavefronts fill every CU at full occupancy (32 wavefronts) several times
// over, as many loads in flight as one voxel per thread gives, with an
// eighth of the partials for the finalize to read.
constexpr int kVarPartBlocks = 8192;
constexpr int kFinThreads = 1024;     // the finalize's one block

__device__ __forceinline__ float soft_d(float z, double tau)
{
    const double m = fabs((double)z) - tau;
    return m > 0.0 ? copysignf((float)m, z) : 0.0f;
}

struct VarArgs {
    Dims d;
    int variant, P;           // P: planes of y1 (2 or 4)
    float gu, gt, gy, omega;  // step sizes, balance
    float mu_lo, mu_hi;
    const float *v;
    VarScalars *sc;
    float *u[2], *t[2];       // ping-pong by iteration parity
    float *s, *y1, *y3, *q, *zs, *zt;
    double *part;             // 2 kVarPartBlocks primal partials, then kVarPartBlocks of r^2
    SelState *sel;
    Hist *hist;
};

// voxel index -> (k, i, j); N < 2^31
__device__ __forceinline__ void coords(const Dims &d, int64_t q, int &k, int &i, int &j)
{
    const uint32_t x = (uint32_t)q, n2 = (uint32_t)d.n2, n1 = (uint32_t)d.n1;
    const uint32_t r = x / n2;
    j = (int)(x - r * n2);
    k = (int)(r / n1);
    i = (int)(r - (uint32_t)k * n1);
}

// (D^T p)(k, i, j) for the vertical plane pv and horizontal plane ph
__device__ __forceinline__ float dT(const Dims &d, const float *pv, const float *ph, int k, int i, int j)
{
    const int64_t q = vox(d, k, i, j);
    float a = 0.f;
    if (i >= 1) a += pv[q - d.n2];
    if (i <= d.n1 - 2) a -= pv[q];
    if (j >= 1) a += ph[q - 1];
    if (j <= d.n2 - 2) a -= ph[q];
    return a;
}

__global__ __launch_bounds__(VT) void k_var_primal(VarArgs a)
{
    __shared__ double red[VT / 64];
    const VarScalars *sc = a.sc;
    if (sc->stop) return;
    const Dims d = a.d;
    const int64_t N = d.plane;
    const int par = (int)(sc->iter & 1u);
    const float *u = a.u[par], *t = a.t[par];
    float *un = a.u[par ^ 1];
    const float a4 = (float)sc->a4;
    const float *y1v = a.y1, *y1h = a.y1 + N;
    double du2 = 0.0, u2 = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * VT + threadIdx.x; q < N; q += (int64_t)gridDim.x * VT) {
        int k, i, j;
        coords(d, q, k, i, j);
        // A^T y1 = D_s^T D^T (first two planes) + omega D^T (the other two)
        float g = 0.f;
        if (k >= 1) g += dT(d, y1v, y1h, k - 1, i, j);
        if (k <= d.n3 - 2) g -= dT(d, y1v, y1h, k, i, j);
        if (a.P == 4) g += a.omega * dT(d, a.y1 + 2 * N, a.y1 + 3 * N, k, i, j);
        const float y4 = a4 * a.q[q];
        const float uo = u[q];
        const float x = uo - a.gu * (g + y4);
        const float nu = fminf(fmaxf(x, a.mu_lo), a.mu_hi);
        un[q] = nu;
        a.zs[q] = a.s[q] - y4;
        float dvt = 0.f;  // (D_v^T y3)(k, i, j)
        if (i >= 1) dvt += a.y3[q - d.n2];
        if (i <= d.n1 - 2) dvt -= a.y3[q];
        a.zt[q] = t[q] - a.gt * (dvt + y4);
        const double dl = (double)nu - (double)uo;
        du2 += dl * dl;
        u2 += (double)uo * (double)uo;
    }
    const double s0 = block_sum<VT>(du2, red);
    const double s1 = block_sum<VT>(u2, red);
    if (threadIdx.x == 0) {
        a.part[2 * blockIdx.x] = s0;
        a.part[2 * blockIdx.x + 1] = s1;
    }
}

// u' = 2 u+ - u at (k, i, j) (the caller keeps the indexes inside the cube)
__device__ __forceinline__ float uprime(const Dims &d, const float *un, const float *uo, int k, int i, int j)
{
    const int64_t q = vox(d, k, i, j);
    return 2.f * un[q] - uo[q];
}

__global__ __launch_bounds__(VT) void k_var_dual(VarArgs a)
{
    __shared__ double red[VT / 64];
    const VarScalars *sc = a.sc;
    if (sc->stop) return;
    const Dims d = a.d;
    const int64_t N = d.plane;
    const int par = (int)(sc->iter & 1u);
    const float *uo = a.u[par], *un = a.u[par ^ 1], *to = a.t[par];
    float *tn = a.t[par ^ 1];
    const double ts = a.sel[0].tau, tt = a.sel[1].tau;
    const float a4 = (float)sc->a4;
    double r2 = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * VT + threadIdx.x; q < N; q += (int64_t)gridDim.x * VT) {
        int k, i, j;
        coords(d, q, k, i, j);
        const float so = a.s[q], sn = soft_d(a.zs[q], ts);
        a.s[q] = sn;
        const float sp = 2.f * sn - so;
        const float tq = soft_d(a.zt[q], tt);
        tn[q] = tq;
        const float tp = 2.f * tq - to[q];
        // y3 += g_y D_v t' (t' one row down from its own z_t and old t)
        if (i <= d.n1 - 2) {
            const float tp1 = 2.f * soft_d(a.zt[q + d.n2], tt) - to[q + d.n2];
            a.y3[q] += a.gy * (tp1 - tp);
        }
        // A u' here: D D_s u' on the edges that exist (and omega D u')
        const float u0 = uprime(d, un, uo, k, i, j);
        const bool ei = i <= d.n1 - 2, ej = j <= d.n2 - 2, ek = k <= d.n3 - 2;
        const float ui = ei ? uprime(d, un, uo, k, i + 1, j) : 0.f;
        const float uj = ej ? uprime(d, un, uo, k, i, j + 1) : 0.f;
        float av[4] = {0.f, 0.f, 0.f, 0.f};
        if (ek) {
            const float s0 = uprime(d, un, uo, k + 1, i, j) - u0;
            if (ei) av[0] = (uprime(d, un, uo, k + 1, i + 1, j) - ui) - s0;
            if (ej) av[1] = (uprime(d, un, uo, k + 1, i, j + 1) - uj) - s0;
        }
        if (ei) av[2] = a.omega * (ui - u0);
        if (ej) av[3] = a.omega * (uj - u0);
        float y[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) y[c] = c < a.P ? a.y1[c * N + q] + a.gy * av[c] : 0.f;
        if (a.variant == GEO_REG_HSSTV2) {
            const float nr = sqrtf((y[0] * y[0] + y[1] * y[1]) + (y[2] * y[2] + y[3] * y[3]));
            if (nr > 1.f) {
#pragma unroll
                for (int c = 0; c < 4; ++c) y[c] = y[c] / nr;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) y[c] = fminf(fmaxf(y[c], -1.f), 1.f);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < a.P) a.y1[c * N + q] = y[c];
        // y4'/g_y - v = (a4/g_y) q + u' + s' + t' - v
        const float qn = (a4 / a.gy) * a.q[q] + ((u0 + sp) + tp) - a.v[q];
        a.q[q] = qn;
        r2 += (double)qn * (double)qn;
    }
    const double tot = block_sum<VT>(r2, red);
    if (threadIdx.x == 0) a.part[2 * kVarPartBlocks + blockIdx.x] = tot;
}

__global__ __launch_bounds__(kFinThreads) void k_var_finalize(VarArgs a, int blocks)
{
    __shared__ double red[kFinThreads / 64];
    VarScalars *sc = a.sc;
    if (sc->stop) return;
    // kFinUnroll partials of each sum in flight per thread (the loads of one
    // round are independent), summed in a fixed order
    constexpr int kFinUnroll = 8;
    double du2 = 0.0, u2 = 0.0, r2 = 0.0;
    for (int b0 = threadIdx.x; b0 < blocks; b0 += kFinUnroll * kFinThreads) {
        double x0[kFinUnroll], x1[kFinUnroll], x2[kFinUnroll];
#pragma unroll
        for (int u = 0; u < kFinUnroll; ++u) {
            const int b = b0 + u * kFinThreads;
            const bool in = b < blocks;
            x0[u] = in ? a.part[2 * b] : 0.0;
            x1[u] = in ? a.part[2 * b + 1] : 0.0;
            x2[u] = in ? a.part[2 * kVarPartBlocks + b] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kFinUnroll; ++u) {
            du2 += x0[u];
            u2 += x1[u];
            r2 += x2[u];
        }
    }
    du2 = block_sum<kFinThreads>(du2, red);
    u2 = block_sum<kFinThreads>(u2, red);
    r2 = block_sum<kFinThreads>(r2, red);
    if (threadIdx.x == 0) {
        const double r = sqrt(r2);
        const double rel = u2 > 0.0 ? sqrt(du2) / sqrt(u2) : __longlong_as_double(0x7ff0000000000000ll);
        const bool bad = !isfinite(du2) || !isfinite(u2) || !isfinite(r2);
        const double c = r > sc->eps ? 1.0 - sc->eps / r : 0.0;
        sc->r = r;
        sc->rel = rel;
        sc->a4 = c * (double)a.gy;
        sc->iter = sc->iter + 1u;
        sc->calls_iter = sc->calls_iter + 1u;
        if (bad) sc->nonfinite = 1u;
        if (bad || (sc->tol > 0.0 && sc->iter >= 2u && rel < sc->tol)) sc->stop = 1u;
    }
}

__global__ __launch_bounds__(VT) void k_var_init(VarArgs a, double eps, double tol)
{
    const int64_t N = a.d.plane;
    for (int64_t q = (int64_t)blockIdx.x * VT + threadIdx.x; q < N; q += (int64_t)gridDim.x * VT) {
        a.u[0][q] = a.v[q];
        a.t[0][q] = 0.f;
        a.s[q] = 0.f;
        a.y3[q] = 0.f;
        a.q[q] = 0.f;
        for (int c = 0; c < a.P; ++c) a.y1[c * N + q] = 0.f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        VarScalars z = {};
        z.eps = eps;
        z.tol = tol;
        *a.sc = z;
    }
}

__global__ void k_var_begin_call(VarScalars *sc, double eps, double tol)
{
    if (threadIdx.x == 0) {
        sc->eps = eps;
        sc->tol = tol;
        sc->calls_iter = 0u;
        sc->stop = sc->nonfinite ? 1u : 0u;
    }
}

// Copy a state variable out (out != null) or in, planes as in the C ABI. A
// loaded y4 is kept as it is, with the factor a4 = 1.
__global__ __launch_bounds__(VT) void k_var_io(VarArgs a, int var, float *out, const float *in)
{
    const int64_t N = a.d.plane;
    const int par = (int)(a.sc->iter & 1u);
    const int64_t n = var == GEO_VAR_Y1 ? a.P * N : N;
    const float a4 = (float)a.sc->a4;
    float *base;
    switch (var) {
    case GEO_VAR_U: base = a.u[par]; break;
    case GEO_VAR_S: base = a.s; break;
    case GEO_VAR_T: base = a.t[par]; break;
    case GEO_VAR_Y1: base = a.y1; break;
    case GEO_VAR_Y3: base = a.y3; break;
    default: base = a.q; break;
    }
    for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) {
        if (out)
            out[g] = var == GEO_VAR_Y4 ? a4 * base[g] : base[g];
        else
            base[g] = in[g];
    }
}

__global__ void k_var_loaded_y4(VarScalars *sc)
{
    if (threadIdx.x == 0) sc->a4 = 1.0;
}

int var_grid(int64_t n)
{
    const int64_t b = (n + VT - 1) / VT;
    return (int)(b < 1 ? 1 : (b > kVarPartBlocks ? kVarPartBlocks : b));
}

size_t align256v(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace: the scalars, partials, search state, then the N-float arrays.
struct VarLayout {
    size_t sc, part, sel, hist, u0, u1, t0, t1, s, y1, y3, q, zs, zt, total;
};

VarLayout var_layout(int64_t N, int P)
{
    VarLayout L;
    size_t o = 0;
    auto take = [&](size_t b) { const size_t at = o; o = align256v(o + b); return at; };
    const size_t f = sizeof(float) * (size_t)N;
    L.sc = take(sizeof(VarScalars));
    L.part = take(sizeof(double) * 3 * kVarPartBlocks);
    L.sel = take(2 * sizeof(SelState));
    L.hist = take(2 * sizeof(Hist));
    L.u0 = take(f);
    L.u1 = take(f);
    L.t0 = take(f);
    L.t1 = take(f);
    L.s = take(f);
    L.y1 = take((size_t)P * f);
    L.y3 = take(f);
    L.q = take(f);
    L.zs = take(f);
    L.zt = take(f);
    L.total = o;
    return L;
}

VarArgs var_args(const Dims &d, const geo_params *p, const float *v, void *ws)
{
    VarArgs a;
    memset(&a, 0, sizeof a);
    a.d = d;
    a.variant = p->regularizer;
    a.P = var_planes(p->regularizer);
    const VarLayout L = var_layout(d.plane, a.P);
    char *b = (char *)ws;
    const double na2 = p->regularizer == GEO_REG_SSTV ? 32.0 : 32.0 + 8.0 * p->omega * p->omega;
    a.gu = (float)(1.0 / (na2 + 1.0));
    a.gt = (float)(1.0 / 5.0);
    a.gy = (float)(1.0 / 3.0);
    a.omega = (float)p->omega;
    a.mu_lo = (float)p->mu_lo;
    a.mu_hi = (float)p->mu_hi;
    a.v = v;
    a.sc = (VarScalars *)(b + L.sc);
    a.part = (double *)(b + L.part);
    a.sel = (SelState *)(b + L.sel);
    a.hist = (Hist *)(b + L.hist);
    a.u[0] = (float *)(b + L.u0);
    a.u[1] = (float *)(b + L.u1);
    a.t[0] = (float *)(b + L.t0);
    a.t[1] = (float *)(b + L.t1);
    a.s = (float *)(b + L.s);
    a.y1 = (float *)(b + L.y1);
    a.y3 = (float *)(b + L.y3);
    a.q = (float *)(b + L.q);
    a.zs = (float *)(b + L.zs);
    a.zt = (float *)(b + L.zt);
    return a;
}

}  // namespace

int var_planes(int regularizer) { return regularizer == GEO_REG_SSTV ? 2 : 4; }

size_t var_workspace_bytes(int n1, int n2, int n3, int regularizer)
{
    return var_layout((int64_t)n1 * n2 * n3, var_planes(regularizer)).total;
}

hipError_t var_state_init(const Dims &d, const geo_params *p, const float *v, void *ws, hipStream_t st)
{
    const VarArgs a = var_args(d, p, v, ws);
    hipLaunchKernelGGL(k_var_init, dim3(var_grid(d.plane)), dim3(VT), 0, st, a, p->eps, p->tol);
    return hipGetLastError();
}

hipError_t var_step(const Dims &d, const geo_params *p, const float *v, void *ws, int n_iter,
                    hipStream_t st, VarScalars *out, double *tau_s, double *tau_t, double *dual_ms)
{
    const VarArgs a = var_args(d, p, v, ws);
    const int G = var_grid(d.plane);
    // dual_ms: events around the dual kernel of every kVarTimedEvery-th
    // iteration from that one on (all of them in calls of fewer), the sampled
    // times scaled to the call
    constexpr int kVarTimedEvery = 8;
    const bool all = n_iter < kVarTimedEvery;
    std::vector<hipEvent_t> ev;
    hipError_t e = hipSuccess;
    if (dual_ms) {
        const int ns = all ? n_iter : n_iter / kVarTimedEvery;
        ev.resize(2 * (size_t)ns);
        for (size_t q = 0; q < ev.size() && e == hipSuccess; ++q) e = hipEventCreate(&ev[q]);
        if (e != hipSuccess) ev.clear();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_var_begin_call, dim3(1), dim3(64), 0, st, a.sc, p->eps, p->tol);
        e = hipGetLastError();
    }
    const uint32_t *stop = &a.sc->stop;
    size_t ne = 0;
    for (int it = 0; it < n_iter && e == hipSuccess; ++it) {
        hipLaunchKernelGGL(k_var_primal, dim3(G), dim3(VT), 0, st, a);
        e = select_begin(a.sel, 2, p->alpha, p->beta, a.hist, stop, st);
        if (e == hipSuccess) e = select_run(a.zs, a.zt, 2, d.plane, a.sel, a.hist, stop, st);
        if (e != hipSuccess) break;
        const bool timed = dual_ms && (all || it % kVarTimedEvery == kVarTimedEvery - 1) &&
                           ne + 2 <= ev.size();
        if (timed) e = hipEventRecord(ev[ne], st);
        hipLaunchKernelGGL(k_var_dual, dim3(G), dim3(VT), 0, st, a);
        if (timed && e == hipSuccess) e = hipEventRecord(ev[ne + 1], st);
        ne += timed ? 2 : 0;
        hipLaunchKernelGGL(k_var_finalize, dim3(1), dim3(kFinThreads), 0, st, a, G);
        if (e == hipSuccess) e = hipGetLastError();
    }
    SelState sel[2];
    if (e == hipSuccess) e = hipMemcpyAsync(out, a.sc, sizeof(VarScalars), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sel, a.sel, sizeof sel, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
        *tau_s = sel[0].tau;
        *tau_t = sel[1].tau;
    }
    if (e == hipSuccess && dual_ms) {
        // iterations after the stopping rule held are no-ops: scale by the
        // iterations done
        double sum = 0.0;
        for (size_t q = 0; q + 1 < ne && e == hipSuccess; q += 2) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[q], ev[q + 1]);
            sum += ms;
        }
        const size_t ns = ne / 2;
        *dual_ms = ns ? sum / (double)ns * (double)out->calls_iter : 0.0;
    }
    for (hipEvent_t x : ev) (void)hipEventDestroy(x);
    return e;
}

hipError_t var_state_io(const Dims &d, const geo_params *p, void *ws, int var, float *out,
                        const float *in, hipStream_t st)
{
    const VarArgs a = var_args(d, p, nullptr, ws);
    const int64_t n = var == GEO_VAR_Y1 ? a.P * d.plane : d.plane;
    hipLaunchKernelGGL(k_var_io, dim3(var_grid(n)), dim3(VT), 0, st, a, var, out, in);
    if (in && var == GEO_VAR_Y4) hipLaunchKernelGGL(k_var_loaded_y4, dim3(1), dim3(64), 0, st, a.sc);
    return hipGetLastError();
}

}  // namespace geo
