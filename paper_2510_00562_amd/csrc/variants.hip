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
// One launch slot per iteration, on the caller's stream, over a one-entry
// launch table in the workspace (the layout the main solver's search,
// histogram passes and finalize read):
//   primal kernel: u+ = P_box(u - g_u (A^T y1 + y4)) into the other u buffer,
//                  the inputs z_s = s - y4 and z_t = t - g_t (D_v^T y3 + y4)
//                  of the two l1-ball projections (stored in the iterations
//                  in which a window is likely to miss, for the histogram
//                  passes; otherwise they evaluate them again from the
//                  state), and per block (a "tile" of the search) the window
//                  statistics, the window candidates and the FP64 partials
//                  of the stopping rule;
//   window search and three histogram passes (select.hip, fallback.hip):
//                  the exact thresholds tau_s, tau_t;
//   dual kernel:   s+, t+ (soft thresholds of z_s, z_t, evaluated again from
//                  the state with the primal kernel's operations: y3 and the
//                  y4 residual are ping-ponged, so the rows next to a voxel
//                  still hold their old values), the extrapolations
//                  x' = 2 x+ - x, y1 += g_y A u' and the conjugate prox of the
//                  regularizer (a clip to [-1, 1], or each 4-entry group
//                  scaled into the unit l2 ball), y3 += g_y D_v t', the y4
//                  residual and FP64 partials of its norm;
//   finalize (sweep.hip): the fidelity-ball factor (y4 - g_y P_B(y4/g_y) =
//                  c g_y (y4/g_y - v), c = max(0, 1 - eps/r), applied when y4
//                  is next read), the relative change, the stopping rule, the
//                  next windows.
// The two streaming kernels are plain (grid-stride, the stencils read
// through the caches); no tile fusion.
#include <math.h>
#include <string.h>

#include <vector>

#include "radix.hpp"

namespace geo {

namespace {

// The primal kernel's blocks are the search's tiles: few of them, so that
// the window search scans few slices (with 4096 blocks of 256 threads it
// took 43 instead of 32 us), and no more than the device holds at once
// (primal_grid). The dual kernel runs up to 8192 blocks of 256 threads (228
// instead of 165 us with 2048 blocks of 1024; 4096 blocks: 2% slower).
constexpr int VT = 1024;          // init and copy kernels
constexpr int VTP = 512;          // primal kernels (68 VGPRs four voxels per thread, 56 one)
constexpr int VTD = 256;          // dual kernel
constexpr int kVarTiles = 768;    // most primal kernel blocks (the workspace regions of the tiles)
constexpr int kVarBBlocks = 8192; // dual kernel blocks

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
    DevScalars *sc;
    float *u[2], *t[2];       // ping-pong by iteration parity
    float *y3[2], *q[2];      // also (the dual kernel reads the rows next to its own)
    float *s, *y1;
    float *z;                 // [2][N]: z_s, z_t (read by the histogram passes)
    double *part;             // [2 * ntiles] primal partials, then [nb] of r^2
    double *winpart;          // [2][ntiles][3]
    float *cand;              // [2][ntiles][capt]
    uint32_t *ccount;         // [2][ntiles]
    const FbRec *rec;
    int ntiles, nb, capt;
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

// The inputs z_s = s - y4 and z_t = t - g_t (D_v^T y3 + y4) of the two
// l1-ball projections, y4 = a4 q, come from y4_of, zs_of and zt_of (with
// the step g_t), the operations every kernel that evaluates them uses: the
// primal and dual kernels here and the histogram passes of a missed window,
// so the values are bit-identical wherever they are evaluated.

// Sums of 8 FP64 values over a block of NT threads in a fixed order; valid
// in thread 0.
template <int NT>
__device__ __forceinline__ void block_sum8v(double (&x)[8], double *red /* 8 * NT/64 */)
{
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = wave_sum(x[c]);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < 8; ++c) red[c * (NT / 64) + wid] = x[c];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            double t = 0.0;
            for (int w = 0; w < NT / 64; ++w) t += red[c * (NT / 64) + w];
            x[c] = t;
        }
}

__global__ __launch_bounds__(VTP) void k_var_primal(VarArgs a)
{
    __shared__ double red[8 * (VTP / 64)];
    __shared__ uint32_t ncand[2];
    DevScalars *sc = a.sc;
    if (idle(sc)) return;
    const Dims d = a.d;
    const int64_t N = d.plane;
    const int tid = threadIdx.x, b = blockIdx.x, nt = a.ntiles;
    if (tid < 2) ncand[tid] = 0u;
    const int par = (int)(sc->iter & 1u);
    const float *u = a.u[par], *t = a.t[par], *y3 = a.y3[par], *qo = a.q[par];
    float *un = a.u[par ^ 1];
    const float a4 = (float)sc->a4;
    const bool zst = sc->zstore != 0u;  // z kept for the histogram passes
    const float *y1v = a.y1, *y1h = a.y1 + N;
    float wlo[2], whi[2];
    bool won[2];
    for (int f = 0; f < 2; ++f) {
        won[f] = sc->sel[f].win_on != 0u;
        wlo[f] = sc->sel[f].win_lo;
        whi[f] = sc->sel[f].win_hi;
    }
    __syncthreads();  // ncand cleared
    double du2 = 0.0, u2 = 0.0, s_hi[2] = {0.0, 0.0}, s_all[2] = {0.0, 0.0};
    float c_hi[2] = {0.f, 0.f};
    // the same trip count for every lane of the block, so that whole
    // wavefronts append candidates
    for (int64_t q0 = (int64_t)b * VTP; q0 < N; q0 += (int64_t)nt * VTP) {
        const int64_t q = q0 + tid;
        const bool in = q < N;
        float z[2] = {0.f, 0.f};
        if (in) {
            int k, i, j;
            coords(d, q, k, i, j);
            // A^T y1 = D_s^T D^T (first two planes) + omega D^T (the other two)
            float g = 0.f;
            if (k >= 1) g += dT(d, y1v, y1h, k - 1, i, j);
            if (k <= d.n3 - 2) g -= dT(d, y1v, y1h, k, i, j);
            if (a.P == 4) g += a.omega * dT(d, a.y1 + 2 * N, a.y1 + 3 * N, k, i, j);
            const float y4 = y4_of(qo[q], a4);
            const float uo = u[q];
            const float x = uo - a.gu * (g + y4);
            const float nu = fminf(fmaxf(x, a.mu_lo), a.mu_hi);
            un[q] = nu;
            const float y3m = i >= 1 ? y3[q - d.n2] : 0.f, y3c = i <= d.n1 - 2 ? y3[q] : 0.f;
            z[0] = zs_of(a.s[q], y4);
            z[1] = zt_of(t[q], y3m, y3c, y4, a.gt);
            if (zst) {
                a.z[q] = z[0];
                a.z[N + q] = z[1];
            }
            const double dl = (double)nu - (double)uo;
            du2 += dl * dl;
            u2 += (double)uo * (double)uo;
        }
        // the window statistics and candidates of the threshold search
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const float av = fabsf(z[f]);
            bool cand = false;
            if (in) {
                s_all[f] += (double)av;
                if (won[f]) {
                    if (av > whi[f]) {
                        c_hi[f] += 1.f;
                        s_hi[f] += (double)av;
                    } else if (av >= wlo[f]) {
                        cand = true;
                    }
                }
            }
            wave_append(cand, av, a.cand + ((int64_t)f * nt + b) * a.capt, &ncand[f], a.capt);
        }
    }
    double acc[8] = {du2, u2, (double)c_hi[0], s_hi[0], s_all[0], (double)c_hi[1], s_hi[1], s_all[1]};
    block_sum8v<VTP>(acc, red);
    if (tid == 0) {
        a.ccount[b] = ncand[0];
        a.ccount[nt + b] = ncand[1];
        a.part[2 * b] = acc[0];
        a.part[2 * b + 1] = acc[1];
        for (int f = 0; f < 2; ++f)
            for (int c = 0; c < 3; ++c) a.winpart[((int64_t)f * nt + b) * 3 + c] = acc[2 + 3 * f + c];
    }
}

// ---- four voxels per thread along j (cubes with N2 % 4 == 0) ----
// The same arithmetic as the kernels above, element by element in the same
// order; whole 16-byte loads and stores of every array, the j - 1 and
// j + 4 neighbours from one more scalar load.
struct F4 {
    float x[4];
};
__device__ __forceinline__ F4 ld4(const float *p)
{
    const float4 v = *reinterpret_cast<const float4 *>(p);
    return F4{{v.x, v.y, v.z, v.w}};
}
__device__ __forceinline__ void st4(float *p, const F4 &v)
{
    *reinterpret_cast<float4 *>(p) = make_float4(v.x[0], v.x[1], v.x[2], v.x[3]);
}

// (D^T p)(k, i, j0 + e), e = 0..3, for the planes pv, ph
__device__ __forceinline__ void dT4(const Dims &d, const float *pv, const float *ph, int k, int i, int j0,
                                    float (&a)[4])
{
    const int64_t q = vox(d, k, i, j0);
    F4 up = {{0.f, 0.f, 0.f, 0.f}}, cv = up;
    if (i >= 1) up = ld4(pv + q - d.n2);
    if (i <= d.n1 - 2) cv = ld4(pv + q);
    const F4 h = ld4(ph + q);
    const float hl = j0 >= 1 ? ph[q - 1] : 0.f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int j = j0 + e;
        float x = 0.f;
        if (i >= 1) x += up.x[e];
        if (i <= d.n1 - 2) x -= cv.x[e];
        if (j >= 1) x += e ? h.x[e - 1] : hl;
        if (j <= d.n2 - 2) x -= h.x[e];
        a[e] = x;
    }
}

__global__ __launch_bounds__(VTP) void k_var_primal4(VarArgs a)
{
    __shared__ double red[8 * (VTP / 64)];
    __shared__ uint32_t ncand[2];
    DevScalars *sc = a.sc;
    if (idle(sc)) return;
    const Dims d = a.d;
    const int64_t N = d.plane, Q = N / 4;
    const int tid = threadIdx.x, b = blockIdx.x, nt = a.ntiles;
    if (tid < 2) ncand[tid] = 0u;
    const int par = (int)(sc->iter & 1u);
    const float *u = a.u[par], *t = a.t[par], *y3 = a.y3[par], *qo = a.q[par];
    float *un = a.u[par ^ 1];
    const float a4 = (float)sc->a4;
    const bool zst = sc->zstore != 0u;  // z kept for the histogram passes
    const float *y1v = a.y1, *y1h = a.y1 + N;
    float wlo[2], whi[2];
    bool won[2];
    for (int f = 0; f < 2; ++f) {
        won[f] = sc->sel[f].win_on != 0u;
        wlo[f] = sc->sel[f].win_lo;
        whi[f] = sc->sel[f].win_hi;
    }
    __syncthreads();  // ncand cleared
    double du2 = 0.0, u2 = 0.0, s_hi[2] = {0.0, 0.0}, s_all[2] = {0.0, 0.0};
    float c_hi[2] = {0.f, 0.f};
    for (int64_t g0 = (int64_t)b * VTP; g0 < Q; g0 += (int64_t)nt * VTP) {
        const int64_t g = g0 + tid;
        const bool in = g < Q;
        float z[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        if (in) {
            const int64_t q = 4 * g;
            int k, i, j0;
            coords(d, q, k, i, j0);
            float gm[4] = {0.f, 0.f, 0.f, 0.f}, gk[4] = {0.f, 0.f, 0.f, 0.f}, go[4] = {0.f, 0.f, 0.f, 0.f};
            if (k >= 1) dT4(d, y1v, y1h, k - 1, i, j0, gm);
            if (k <= d.n3 - 2) dT4(d, y1v, y1h, k, i, j0, gk);
            if (a.P == 4) dT4(d, a.y1 + 2 * N, a.y1 + 3 * N, k, i, j0, go);
            const F4 qv = ld4(qo + q), uo = ld4(u + q), sv = ld4(a.s + q), tv = ld4(t + q);
            F4 y3m = {{0.f, 0.f, 0.f, 0.f}}, y3c = y3m;
            if (i >= 1) y3m = ld4(y3 + q - d.n2);
            if (i <= d.n1 - 2) y3c = ld4(y3 + q);
            F4 nu, zs, zt;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float gg = 0.f;
                if (k >= 1) gg += gm[e];
                if (k <= d.n3 - 2) gg -= gk[e];
                if (a.P == 4) gg += a.omega * go[e];
                const float y4 = y4_of(qv.x[e], a4);
                const float x = uo.x[e] - a.gu * (gg + y4);
                nu.x[e] = fminf(fmaxf(x, a.mu_lo), a.mu_hi);
                zs.x[e] = zs_of(sv.x[e], y4);
                zt.x[e] = zt_of(tv.x[e], y3m.x[e], y3c.x[e], y4, a.gt);
                z[0][e] = zs.x[e];
                z[1][e] = zt.x[e];
                const double dl = (double)nu.x[e] - (double)uo.x[e];
                du2 += dl * dl;
                u2 += (double)uo.x[e] * (double)uo.x[e];
            }
            st4(un + q, nu);
            if (zst) {
                st4(a.z + q, zs);
                st4(a.z + N + q, zt);
            }
        }
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float av = fabsf(z[f][e]);
                bool cand = false;
                if (in) {
                    s_all[f] += (double)av;
                    if (won[f]) {
                        if (av > whi[f]) {
                            c_hi[f] += 1.f;
                            s_hi[f] += (double)av;
                        } else if (av >= wlo[f]) {
                            cand = true;
                        }
                    }
                }
                wave_append(cand, av, a.cand + ((int64_t)f * nt + b) * a.capt, &ncand[f], a.capt);
            }
    }
    double acc[8] = {du2, u2, (double)c_hi[0], s_hi[0], s_all[0], (double)c_hi[1], s_hi[1], s_all[1]};
    block_sum8v<VTP>(acc, red);
    if (tid == 0) {
        a.ccount[b] = ncand[0];
        a.ccount[nt + b] = ncand[1];
        a.part[2 * b] = acc[0];
        a.part[2 * b + 1] = acc[1];
        for (int f = 0; f < 2; ++f)
            for (int c = 0; c < 3; ++c) a.winpart[((int64_t)f * nt + b) * 3 + c] = acc[2 + 3 * f + c];
    }
}

// u' = 2 u+ - u at (k, i, j) (the caller keeps the indexes inside the cube)
__device__ __forceinline__ float uprime(const Dims &d, const float *un, const float *uo, int k, int i, int j)
{
    const int64_t q = vox(d, k, i, j);
    return 2.f * un[q] - uo[q];
}

__global__ __launch_bounds__(VTD) void k_var_dual(VarArgs a)
{
    __shared__ double red[VTD / 64];
    const DevScalars *sc = a.sc;
    if (idle(sc)) return;
    const Dims d = a.d;
    const int64_t N = d.plane;
    const int par = (int)(sc->iter & 1u);
    const float *uo = a.u[par], *un = a.u[par ^ 1], *to = a.t[par];
    const float *y3o = a.y3[par], *qo = a.q[par];
    float *tn = a.t[par ^ 1], *y3n = a.y3[par ^ 1], *qn = a.q[par ^ 1];
    // the thresholds: from the window search, or from this slot's passes
    const double ts = sc->sel[0].done ? sc->sel[0].tau : fb_final(a.rec, 0).tau;
    const double tt = sc->sel[1].done ? sc->sel[1].tau : fb_final(a.rec, 1).tau;
    const float a4 = (float)sc->a4;
    double r2 = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * VTD + threadIdx.x; q < N; q += (int64_t)gridDim.x * VTD) {
        int k, i, j;
        coords(d, q, k, i, j);
        // z_s, z_t here as the primal kernel evaluated them
        const float y4 = y4_of(qo[q], a4), y3c = y3o[q];
        const float y3m = i >= 1 ? y3o[q - d.n2] : 0.f;
        const float so = a.s[q], sn = soft_d(zs_of(so, y4), ts);
        a.s[q] = sn;
        const float sp = 2.f * sn - so;
        const float tq = soft_d(zt_of(to[q], y3m, i <= d.n1 - 2 ? y3c : 0.f, y4, a.gt), tt);
        tn[q] = tq;
        const float tp = 2.f * tq - to[q];
        // y3 += g_y D_v t' (t' one row down from its own z_t and old t); the
        // last row keeps its value
        float y3x = y3c;
        if (i <= d.n1 - 2) {
            const int64_t qd = q + d.n2;
            const float y4d = y4_of(qo[qd], a4), y3d = i + 1 <= d.n1 - 2 ? y3o[qd] : 0.f;
            const float ztd = zt_of(to[qd], y3c, y3d, y4d, a.gt);
            const float tp1 = 2.f * soft_d(ztd, tt) - to[qd];
            y3x = y3c + a.gy * (tp1 - tp);
        }
        y3n[q] = y3x;
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
        const float qx = (a4 / a.gy) * qo[q] + ((u0 + sp) + tp) - a.v[q];
        qn[q] = qx;
        r2 += (double)qx * (double)qx;
    }
    const double tot = block_sum<VTD>(r2, red);
    if (threadIdx.x == 0) a.part[2 * a.ntiles + blockIdx.x] = tot;
}

// u' = 2 u+ - u at four voxels from (k, i, j0), and at (k, i, j0 + 4)
__device__ __forceinline__ void uprime4(const Dims &d, const float *un, const float *uo, int k, int i, int j0,
                                        F4 &up, float &next)
{
    const int64_t q = vox(d, k, i, j0);
    const F4 a = ld4(un + q), b = ld4(uo + q);
#pragma unroll
    for (int e = 0; e < 4; ++e) up.x[e] = 2.f * a.x[e] - b.x[e];
    next = j0 + 4 < d.n2 ? 2.f * un[q + 4] - uo[q + 4] : 0.f;
}

__global__ __launch_bounds__(VTD) void k_var_dual4(VarArgs a)
{
    __shared__ double red[VTD / 64];
    const DevScalars *sc = a.sc;
    if (idle(sc)) return;
    const Dims d = a.d;
    const int64_t N = d.plane, Q = N / 4;
    const int par = (int)(sc->iter & 1u);
    const float *uo = a.u[par], *un = a.u[par ^ 1], *to = a.t[par];
    const float *y3o = a.y3[par], *qo = a.q[par];
    float *tn = a.t[par ^ 1], *y3n = a.y3[par ^ 1], *qw = a.q[par ^ 1];
    const double ts = sc->sel[0].done ? sc->sel[0].tau : fb_final(a.rec, 0).tau;
    const double tt = sc->sel[1].done ? sc->sel[1].tau : fb_final(a.rec, 1).tau;
    const float a4 = (float)sc->a4;
    double r2 = 0.0;
    for (int64_t g = (int64_t)blockIdx.x * VTD + threadIdx.x; g < Q; g += (int64_t)gridDim.x * VTD) {
        const int64_t q = 4 * g;
        int k, i, j0;
        coords(d, q, k, i, j0);
        const bool ei = i <= d.n1 - 2, ek = k <= d.n3 - 2;
        const F4 so = ld4(a.s + q), tov = ld4(to + q), qv = ld4(qo + q), y3c = ld4(y3o + q);
        F4 y3m = {{0.f, 0.f, 0.f, 0.f}};
        if (i >= 1) y3m = ld4(y3o + q - d.n2);
        F4 sn, tq, sp, tp;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // z_s, z_t here as the primal kernel evaluated them
            const float y4 = y4_of(qv.x[e], a4);
            sn.x[e] = soft_d(zs_of(so.x[e], y4), ts);
            sp.x[e] = 2.f * sn.x[e] - so.x[e];
            tq.x[e] = soft_d(zt_of(tov.x[e], y3m.x[e], ei ? y3c.x[e] : 0.f, y4, a.gt), tt);
            tp.x[e] = 2.f * tq.x[e] - tov.x[e];
        }
        st4(a.s + q, sn);
        st4(tn + q, tq);
        // y3 += g_y D_v t' (t' one row down from its own z_t and old t); the
        // last row keeps its value
        F4 y3x = y3c;
        if (ei) {
            const int64_t qd = q + d.n2;
            const F4 td = ld4(to + qd), qd4 = ld4(qo + qd);
            F4 y3d = {{0.f, 0.f, 0.f, 0.f}};
            if (i + 1 <= d.n1 - 2) y3d = ld4(y3o + qd);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float ztd = zt_of(td.x[e], y3c.x[e], y3d.x[e], y4_of(qd4.x[e], a4), a.gt);
                const float tp1 = 2.f * soft_d(ztd, tt) - td.x[e];
                y3x.x[e] = y3c.x[e] + a.gy * (tp1 - tp.x[e]);
            }
        }
        st4(y3n + q, y3x);
        // u' on the rows (k, i), (k, i + 1), (k + 1, i), (k + 1, i + 1)
        F4 u0, ui = {{0.f, 0.f, 0.f, 0.f}}, uk = ui, uki = ui;
        float u0n, ukn = 0.f, dummy;
        uprime4(d, un, uo, k, i, j0, u0, u0n);
        if (ei) uprime4(d, un, uo, k, i + 1, j0, ui, dummy);
        if (ek) uprime4(d, un, uo, k + 1, i, j0, uk, ukn);
        if (ek && ei) uprime4(d, un, uo, k + 1, i + 1, j0, uki, dummy);
        F4 yv[4];
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < a.P) yv[c] = ld4(a.y1 + c * N + q);
        const F4 vv = ld4(a.v + q);
        F4 qn;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool ej = j0 + e <= d.n2 - 2;
            const float uj = ej ? (e < 3 ? u0.x[e + 1] : u0n) : 0.f;
            float av[4] = {0.f, 0.f, 0.f, 0.f};
            if (ek) {
                const float s0 = uk.x[e] - u0.x[e];
                if (ei) av[0] = (uki.x[e] - ui.x[e]) - s0;
                if (ej) av[1] = ((e < 3 ? uk.x[e + 1] : ukn) - uj) - s0;
            }
            if (ei) av[2] = a.omega * (ui.x[e] - u0.x[e]);
            if (ej) av[3] = a.omega * (uj - u0.x[e]);
            float y[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) y[c] = c < a.P ? yv[c].x[e] + a.gy * av[c] : 0.f;
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
            for (int c = 0; c < 4; ++c) yv[c].x[e] = y[c];
            qn.x[e] = (a4 / a.gy) * qv.x[e] + ((u0.x[e] + sp.x[e]) + tp.x[e]) - vv.x[e];
            r2 += (double)qn.x[e] * (double)qn.x[e];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < a.P) st4(a.y1 + c * N + q, yv[c]);
        st4(qw + q, qn);
    }
    const double tot = block_sum<VTD>(r2, red);
    if (threadIdx.x == 0) a.part[2 * a.ntiles + blockIdx.x] = tot;
}

__global__ __launch_bounds__(VT) void k_var_init(VarArgs a, double eps, double tol, double alpha,
                                                 double beta, double gy4)
{
    const int64_t N = a.d.plane;
    for (int64_t q = (int64_t)blockIdx.x * VT + threadIdx.x; q < N; q += (int64_t)gridDim.x * VT) {
        a.u[0][q] = a.v[q];
        a.t[0][q] = 0.f;
        a.s[q] = 0.f;
        a.y3[0][q] = 0.f;
        a.q[0][q] = 0.f;
        for (int c = 0; c < a.P; ++c) a.y1[c * N + q] = 0.f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevScalars z = {};
        z.c4 = 1.0;
        z.a4 = 1.0;
        z.eps = eps;
        z.tol = tol;
        z.sel[0].radius = alpha;
        z.sel[1].radius = beta;
        z.sel[0].done = z.sel[1].done = 1u;  // no search pending
        z.zstore = 1u;
        z.gy4 = gy4;
        *a.sc = z;
    }
}

__global__ void k_var_begin_call(DevScalars *sc, double eps, double tol, double alpha, double beta,
                                 uint32_t limit)
{
    if (threadIdx.x == 0) {
        sc->eps = eps;
        sc->tol = tol;
        sc->calls_iter = 0u;
        sc->call_limit = limit;
        sc->fallback = 0u;
        sc->sel[0].radius = alpha;
        sc->sel[1].radius = beta;
        sc->stop = sc->nonfinite ? 1u : 0u;
    }
}

// Copy a state variable out (out != null) or in, planes as in the C ABI.
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
    case GEO_VAR_Y3: base = a.y3[par]; break;
    default: base = a.q[par]; break;
    }
    for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) {
        if (out)
            out[g] = var == GEO_VAR_Y4 ? a4 * base[g] : base[g];
        else
            base[g] = in[g];  // a loaded y4 is kept as it is, with the factor 1
    }
}

int grid_of(int64_t n, int cap, int threads = VT)
{
    const int64_t b = (n + threads - 1) / threads;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

size_t align256v(size_t x) { return (x + 255) & ~(size_t)255; }

// Blocks of `kernel` that the device holds at once (queried once per kernel).
template <typename K>
int resident_blocks(K kernel, int threads)
{
    int dev = 0, cus = 256, per = 1;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per < 1)
        per = 1;
    return cus * per;
}

// Primal kernel blocks for N voxels: enough for one voxel (or group of four)
// per thread, at most what the device holds at once (three blocks per CU of
// the four-voxel kernel, four of the one-voxel kernel) and kVarTiles (three
// per CU of 256), so that the grid runs in one round: 1024 blocks of the
// four-voxel kernel left a second round of 256 (iterations 2.4% (HSSTV2)
// and 3.2% (SSTV) slower than with 768; with 512, 1.2% and 2.4%). The
// workspace regions of the tiles sized for 1024 instead of 768 moved the
// arrays after them and made the dual kernel 2% slower.
int primal_grid(int64_t N, bool quads)
{
    static const int res1 = resident_blocks(k_var_primal, VTP), res4 = resident_blocks(k_var_primal4, VTP);
    const int cap = quads ? res4 : res1;
    return grid_of(quads ? N / 4 : N, cap < kVarTiles ? cap : kVarTiles, VTP);
}

// four voxels per thread when rows split into whole 16-byte groups and v is
// 16-byte aligned (the workspace arrays are 256-byte aligned)
bool use_quads(const Dims &d, const float *v) { return d.n2 % 4 == 0 && ((uintptr_t)v & 15u) == 0; }

// Workspace: the scalars, the search's regions, the launch table, then the
// N-float arrays.
struct VarLayout {
    size_t sc, part, winpart, hist, rec, cand, ccount, table, u0, u1, t0, t1, s, y1, y3[2], q[2], z, total;
    int max_tiles, nb;  // most primal blocks, dual blocks
    int64_t cap;        // candidates per field
};

VarLayout var_layout(int64_t N, int P)
{
    VarLayout L;
    L.max_tiles = grid_of(N, kVarTiles, VTP);
    L.nb = grid_of(N, kVarBBlocks, VTD);
    L.cap = N / 16 > 65536 ? N / 16 : 65536;
    size_t o = 0;
    auto take = [&](size_t b) { const size_t at = o; o = align256v(o + b); return at; };
    const size_t f = sizeof(float) * (size_t)N;
    L.sc = take(sizeof(DevScalars));
    L.part = take(sizeof(double) * (2 * (size_t)L.max_tiles + (size_t)L.nb));
    L.winpart = take(sizeof(double) * 2 * 3 * (size_t)L.max_tiles);
    L.hist = take(6 * sizeof(Hist));  // 3 radix levels x 2 fields
    L.rec = take(6 * sizeof(FbRec));
    L.cand = take(sizeof(float) * 2 * (size_t)L.cap);
    L.ccount = take(sizeof(uint32_t) * 2 * (size_t)L.max_tiles);
    L.table = take(table_bytes(1));
    L.u0 = take(f);
    L.u1 = take(f);
    L.t0 = take(f);
    L.t1 = take(f);
    L.s = take(f);
    L.y1 = take((size_t)P * f);
    L.y3[0] = take(f);
    L.y3[1] = take(f);
    L.q[0] = take(f);
    L.q[1] = take(f);
    L.z = take(2 * f);
    L.total = o;
    return L;
}

VarArgs var_args(const Dims &d, const geo_params *p, const float *v, void *ws, VarLayout *Lout = nullptr)
{
    VarArgs a;
    memset(&a, 0, sizeof a);
    a.d = d;
    a.variant = p->regularizer;
    a.P = var_planes(p->regularizer);
    const VarLayout L = var_layout(d.plane, a.P);
    if (Lout) *Lout = L;
    char *b = (char *)ws;
    const double na2 = p->regularizer == GEO_REG_SSTV ? 32.0 : 32.0 + 8.0 * p->omega * p->omega;
    a.gu = (float)(1.0 / (na2 + 1.0));
    a.gt = (float)(1.0 / 5.0);
    a.gy = (float)(1.0 / 3.0);
    a.omega = (float)p->omega;
    a.mu_lo = (float)p->mu_lo;
    a.mu_hi = (float)p->mu_hi;
    a.v = v;
    a.sc = (DevScalars *)(b + L.sc);
    a.part = (double *)(b + L.part);
    a.winpart = (double *)(b + L.winpart);
    a.cand = (float *)(b + L.cand);
    a.ccount = (uint32_t *)(b + L.ccount);
    a.rec = (const FbRec *)(b + L.rec);
    a.u[0] = (float *)(b + L.u0);
    a.u[1] = (float *)(b + L.u1);
    a.t[0] = (float *)(b + L.t0);
    a.t[1] = (float *)(b + L.t1);
    a.s = (float *)(b + L.s);
    a.y1 = (float *)(b + L.y1);
    a.y3[0] = (float *)(b + L.y3[0]);
    a.y3[1] = (float *)(b + L.y3[1]);
    a.q[0] = (float *)(b + L.q[0]);
    a.q[1] = (float *)(b + L.q[1]);
    a.z = (float *)(b + L.z);
    // the primal grid (at most max_tiles: both forms need at most N / VTP)
    a.ntiles = primal_grid(d.plane, v && use_quads(d, v));
    a.nb = L.nb;
    a.capt = (int)(L.cap / a.ntiles);
    return a;
}

// Host image of the launch table entry: the fields the window search, the
// histogram passes and the finalize read. The tile geometry and the sweep B
// prefetch of the main solver stay zero. The state sides hold the arrays
// from which the histogram passes evaluate z_s and z_t (s, t, y3, the y4
// residual) when the primal kernel did not store them.
void var_table_entry(CubeEntry *e, const VarArgs &a, const VarLayout &L, void *ws)
{
    memset(e, 0, sizeof *e);
    CubeArgs<float> *x = reinterpret_cast<CubeArgs<float> *>(e->bytes);
    char *b = (char *)ws;
    for (int p = 0; p < 2; ++p) {
        x->side[p].s = a.s;
        x->side[p].t = a.t[p];
        x->side[p].y3 = a.y3[p];
        x->side[p].y4 = a.q[p];
    }
    CubeCommon &c = x->c;
    c.zt_step = a.gt;
    c.d = a.d;
    c.v = a.v;
    c.sc = a.sc;
    c.part = a.part;
    c.winpart = a.winpart;
    c.hist = (Hist *)(b + L.hist);
    c.rec = (FbRec *)(b + L.rec);
    c.cand = a.cand;
    c.ccount = a.ccount;
    c.zbuf = a.z;
    c.capt = a.capt;
    c.ntiles = a.ntiles;
    c.nb = a.nb;
    c.mu_lo = a.mu_lo;
    c.mu_hi = a.mu_hi;
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
    // y4 = gy4 c4 q after an iteration, gy4 the FP32 step the kernels use
    hipLaunchKernelGGL(k_var_init, dim3(grid_of(d.plane, kVarBBlocks)), dim3(VT), 0, st, a, p->eps,
                       p->tol, p->alpha, p->beta, (double)a.gy);
    return hipGetLastError();
}

hipError_t var_step(const Dims &d, const geo_params *p, const float *v, void *ws, int n_iter,
                    hipStream_t st, DevScalars *out, int *slots, double *dual_ms)
{
    VarLayout L;
    const VarArgs a = var_args(d, p, v, ws, &L);
    void *table = (char *)ws + L.table;
    const int stride = (int)sizeof(CubeArgs<float>);
    LaunchShape sh;
    memset(&sh, 0, sizeof sh);
    sh.ncubes = 1;
    sh.fb_grid = fallback_grid();
    // the table image, with its launch-wide flags zeroed
    std::vector<unsigned char> img(table_bytes(1), 0);
    var_table_entry(reinterpret_cast<CubeEntry *>(img.data()), a, L, ws);
    hipError_t e = hipMemcpyAsync(table, img.data(), img.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_var_begin_call, dim3(1), dim3(64), 0, st, a.sc, p->eps, p->tol, p->alpha,
                           p->beta, (uint32_t)n_iter);
        e = hipGetLastError();
    }
    // dual_ms: events around the dual kernel of the kTimedEvery-th,
    // 2 kTimedEvery-th, ... slot of the call (every slot in calls of fewer),
    // the mean scaled to the iterations done
    const bool all = n_iter < kTimedEvery;
    std::vector<hipEvent_t> ev;
    if (dual_ms && e == hipSuccess) {
        ev.resize(2 * (size_t)(all ? n_iter : n_iter / kTimedEvery));
        for (size_t k = 0; k < ev.size() && e == hipSuccess; ++k) e = hipEventCreate(&ev[k]);
    }
    const bool quads = use_quads(d, v);
    // with a tolerance the host reads the stop flag every check_every slots
    const int every = p->tol > 0.0 ? (p->check_every > 0 ? p->check_every : 32) : (n_iter > 0 ? n_iter : 1);
    size_t ne = 0;
    int issued = 0;
    bool synced = false;
    while (issued < n_iter && e == hipSuccess) {
        const int batch = n_iter - issued < every ? n_iter - issued : every;
        for (int it = issued; it < issued + batch && e == hipSuccess; ++it) {
            if (quads)
                hipLaunchKernelGGL(k_var_primal4, dim3(a.ntiles), dim3(VTP), 0, st, a);
            else
                hipLaunchKernelGGL(k_var_primal, dim3(a.ntiles), dim3(VTP), 0, st, a);
            e = launch_select_window(table, stride, 1, 0, st);
            for (int level = 0; level < 3 && e == hipSuccess; ++level)
                e = launch_fallback(table, 4, sh, level, st);
            if (e != hipSuccess) break;
            const bool timed = dual_ms && (all || it % kTimedEvery == kTimedEvery - 1) &&
                               ne + 2 <= ev.size();
            if (timed) e = hipEventRecord(ev[ne], st);
            if (quads)
                hipLaunchKernelGGL(k_var_dual4, dim3(a.nb), dim3(VTD), 0, st, a);
            else
                hipLaunchKernelGGL(k_var_dual, dim3(a.nb), dim3(VTD), 0, st, a);
            if (timed && e == hipSuccess) e = hipEventRecord(ev[ne + 1], st);
            ne += timed ? 2 : 0;
            if (e == hipSuccess) e = launch_finalize(table, stride, 1, st);
        }
        issued += batch;
        if (e == hipSuccess) e = hipMemcpyAsync(out, a.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        synced = e == hipSuccess;
        if (synced && (out->stop || (int)out->calls_iter >= n_iter)) break;
    }
    if (!synced && e == hipSuccess) {  // n_iter = 0
        e = hipMemcpyAsync(out, a.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    *slots = issued;
    if (e == hipSuccess && dual_ms) {
        double sum = 0.0;
        for (size_t k = 0; k + 1 < ne && e == hipSuccess; k += 2) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
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
    hipLaunchKernelGGL(k_var_io, dim3(grid_of(n, kVarBBlocks)), dim3(VT), 0, st, a, var, out, in);
    hipError_t e = hipGetLastError();
    // a loaded state does not continue the previous run: y4 read with the
    // factor 1, the threshold predictions dropped
    if (e == hipSuccess && in) e = launch_state_loaded(a.sc, var, st);
    return e;
}

}  // namespace geo
