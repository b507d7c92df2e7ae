// One iteration of Alg. 1 (problem (20)) as HBM-streaming sweeps for gfx950.
//
//   sweep A  (fused, LDS-tiled): steps 1, 4, 5, the extrapolations 6 and 9-10,
//            steps 11 and 12, the u' part of step 14, and the inputs of the
//            two l1-ball projections (z_s of step 2, z_t of step 3) plus the
//            FP64 partial sums of the stopping rule (eq. (28)).
//   select   (select.hip): exact soft-threshold levels tau_s, tau_t.
//   sweep B  (pointwise): steps 2, 3, 7, 8, 13, the rest of step 14 and the
//            FP64 partial sums of the l2-ball distance of step 15.
//   finalize (one block): the l2-ball factor of step 15 (applied lazily when
//            y4 is next read), the stopping test and the iteration counter.
//
// Sweep A keeps the w1/w2 extrapolations (12 of the 21 state words per voxel)
// out of HBM: a workgroup owns a TI x TJ pixel tile and marches through a
// chunk of bands; for each band it stages the masked dual edge fields y1, y2
// with a 2-pixel halo in LDS, recomputes w' on a 1-pixel ring and u' on the
// (i+1, j+1) ring, and updates y1, y2 from LDS. The D_s coupling between bands
// is carried in LDS from one band to the next.
//
// Every state array is ping-ponged: iteration k reads side (k & 1) and writes
// side ((k + 1) & 1), so halo reads never race with writes. The side is taken
// from the device iteration counter, which makes one iteration's launches a
// fixed sequence (and the stopping rule a device flag that turns the rest of
// the launches into no-ops, so iteration counts stay exact).
#include "solver.hpp"

namespace geo {

namespace {

constexpr int TI = kTI, TJ = kTJ, KC = kKC, NT = kSweepThreads;
constexpr int H2 = TI + 4, W2 = TJ + 4, S2 = H2 * W2;  // y halo 2
constexpr int H1 = TI + 2, W1 = TJ + 2, S1 = H1 * W1;  // w' ring 1
constexpr int HU = TI + 1, WU = TJ + 1, SU = HU * WU;  // u' ring (+1, +1)

template <typename DT>
struct IterArgs {
    Dims d;
    const float *v;
    Side<DT> side[2];
    DT *y4p;  // y4 + u'/5 (step 14, first part)
    float *zs, *zt;
    DevScalars *sc;
    double *part;  // [blocks_a * 2 | blocks_b]
    int blocks_a;
    SweepGrid g;
    float thr1;  // omega * step_w1
    float mu_lo, mu_hi;
};

// Block -> tile. Workgroups are dispatched round-robin over the 8 XCDs; give
// each XCD a contiguous run of tiles (j fastest, then i, then band chunk) so
// that halo rows shared by neighbouring tiles meet in the same L2.
__device__ __forceinline__ void tile_of(const SweepGrid &g, int &tj, int &ti, int &tk)
{
    const int nb = g.tj * g.ti * g.tk;
    const int b = blockIdx.x;
    int t = b;
    if (nb >= 64) {
        const int xcd = b & 7, slot = b >> 3;
        const int per = nb >> 3, rem = nb & 7;
        // XCDs 0..rem-1 own per+1 tiles, the rest per tiles
        t = xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
    }
    tj = t % g.tj;
    const int r = t / g.tj;
    ti = r % g.ti;
    tk = r / g.ti;
}

template <typename DT>
__global__ __launch_bounds__(NT) void k_sweep_a(IterArgs<DT> a)
{
    const DevScalars *sc = a.sc;
    if (sc->stop) return;
    __shared__ float sY[2][4][S2];  // [band parity][y1v, y1h, y2v, y2h] masked
    __shared__ float sU[2][SU];     // u' by band parity
    __shared__ float sW[2][6][S1];  // w1', w2' (masked ud/lr planes)
    __shared__ double red[NT / 64];

    const Dims d = a.d;
    const int n1 = d.n1, n2 = d.n2, n3 = d.n3;
    const int64_t N = d.plane;
    const int par = (int)(sc->iter & 1u);
    const Side<DT> src = a.side[par], dst = a.side[par ^ 1];
    const float c4 = (float)sc->c4, d4v = (float)(sc->d4 * 0.2);
    int tj, ti, tk;
    tile_of(a.g, tj, ti, tk);
    const int j0 = tj * TJ, i0 = ti * TI, kb = tk * KC;
    const int ke = min(kb + KC, n3);
    const int tid = threadIdx.x;
    double du2 = 0.0, u2 = 0.0;

    auto loadY = [&](int k, int buf) {
        for (int p = tid; p < S2; p += NT) {
            const int li = p / W2, lj = p - li * W2;
            const int i = i0 - 2 + li, j = j0 - 2 + lj;
            float a1 = 0.f, b1 = 0.f, a2 = 0.f, b2 = 0.f;
            if (k >= 0 && k < n3 && i >= 0 && i < n1 && j >= 0 && j < n2) {
                const int64_t q = vox(d, k, i, j);
                if (i <= n1 - 2) {
                    a1 = ld(src.y1 + q);
                    a2 = ld(src.y2 + q);
                }
                if (j <= n2 - 2) {
                    b1 = ld(src.y1 + N + q);
                    b2 = ld(src.y2 + N + q);
                }
            }
            sY[buf][0][p] = a1;
            sY[buf][1][p] = b1;
            sY[buf][2][p] = a2;
            sY[buf][3][p] = b2;
        }
    };
    // D^T (y_v, y_h) at R2-local (li, lj) from the masked fields in LDS
    auto dT = [&](int buf, int pv, int li, int lj) {
        const float *yv = sY[buf][pv], *yh = sY[buf][pv + 1];
        const int c = li * W2 + lj;
        return (yv[c - W2] - yv[c]) + (yh[c - 1] - yh[c]);
    };
    // u+ and u' for band kk on the (i+1, j+1) ring; own points also write
    // u+, y4 + u'/5 and the l1-projection inputs z_s, z_t of band kk.
    auto uphase = [&](int kk, bool own_band) {
        const int buf = kk & 1;
        for (int p = tid; p < SU; p += NT) {
            const int ui = p / WU, uj = p - ui * WU;
            const int i = i0 + ui, j = j0 + uj;
            float up = 0.f;
            if (kk < n3 && i < n1 && j < n2) {
                const int li = ui + 2, lj = uj + 2;
                // D^T y1 + D_s^T D^T y2 at band kk
                float g = dT(buf, 0, li, lj);
                if (kk <= n3 - 2) g -= dT(buf, 2, li, lj);
                if (kk >= 1) g += dT(buf ^ 1, 2, li, lj);
                const int64_t q = vox(d, kk, i, j);
                const float vq = a.v[q];
                const float y4 = c4 * (ld(src.y4 + q) - d4v * vq);
                const float uo = src.u[q];
                const float x = uo - kStepU * (g + y4);
                const float un = x < a.mu_lo ? a.mu_lo : (x > a.mu_hi ? a.mu_hi : x);
                up = 2.f * un - uo;
                if (own_band && ui < TI && uj < TJ) {
                    dst.u[q] = un;
                    st(a.y4p + q, y4 + kStepY * up);
                    const float dl = un - uo;
                    du2 += (double)dl * (double)dl;
                    u2 += (double)uo * (double)uo;
                    const float y3c = i <= n1 - 2 ? ld(src.y3 + q) : 0.f;
                    const float y3m = i >= 1 ? ld(src.y3 + q - n2) : 0.f;
                    a.zs[q] = src.s[q] - y4;                          // step 2 (gamma_s = 1)
                    a.zt[q] = src.t[q] - kStepT * ((y3m - y3c) + y4);  // step 3
                }
            }
            sU[buf][p] = up;
        }
    };
    // w1+, w2+ (steps 4, 5) and w' (steps 9, 10) on the 1-pixel ring of band k
    auto wphase = [&](int k) {
        const int buf = k & 1;
        for (int p = tid; p < S1; p += NT) {
            const int wi = p / W1, wj = p - wi * W1;
            const int i = i0 - 1 + wi, j = j0 - 1 + wj;
            const bool in = i >= 0 && i < n1 && j >= 0 && j < n2;
            const bool own = wi >= 1 && wi <= TI && wj >= 1 && wj <= TJ;
            const float mv = mask_le(i, n1), mh = mask_le(j, n2);
            const int c = (wi + 1) * W2 + (wj + 1);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                float o[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                if (in) {
                    const float *yv = sY[buf][2 * f], *yh = sY[buf][2 * f + 1];
                    float L[6];
                    L[0] = mv * yv[c];
                    L[1] = mv * 0.25f * ((yh[c] + yh[c - 1]) + (yh[c + W2] + yh[c + W2 - 1]));
                    L[2] = mh * 0.25f * ((yv[c] + yv[c - W2]) + (yv[c + 1] + yv[c - W2 + 1]));
                    L[3] = mh * yh[c];
                    L[4] = 0.5f * (yv[c] + yv[c - W2]);
                    L[5] = 0.5f * (yh[c] + yh[c - 1]);
                    const int64_t q = vox(d, k, i, j);
                    const float *w = f ? src.w2 : src.w1;
                    float *wd = f ? dst.w2 : dst.w1;
                    const float thr = f ? kStepW : a.thr1;
                    float wo[6], wn[6];
#pragma unroll
                    for (int cc = 0; cc < 6; ++cc) {
                        wo[cc] = w[cc * N + q];
                        wn[cc] = wo[cc] + kStepW * L[cc];
                    }
                    shrink2(wn[0], wn[1], thr);
                    shrink2(wn[2], wn[3], thr);
                    shrink2(wn[4], wn[5], thr);
                    if (own) {
#pragma unroll
                        for (int cc = 0; cc < 6; ++cc) wd[cc * N + q] = wn[cc];
                    }
#pragma unroll
                    for (int cc = 0; cc < 6; ++cc) o[cc] = 2.f * wn[cc] - wo[cc];
                    o[0] *= mv;
                    o[1] *= mv;
                    o[2] *= mh;
                    o[3] *= mh;
                }
#pragma unroll
                for (int cc = 0; cc < 6; ++cc) sW[f][cc][p] = o[cc];
            }
        }
    };
    // y1+, y2+ (steps 11, 12) of band k on the tile
    auto yphase = [&](int k) {
        const float msk = k <= n3 - 2 ? 1.f : 0.f;
        for (int p = tid; p < TI * TJ; p += NT) {
            const int ti_ = p / TJ, tj_ = p - ti_ * TJ;
            const int i = i0 + ti_, j = j0 + tj_;
            if (i >= n1 || j >= n2) continue;
            const float mv = mask_le(i, n1), mh = mask_le(j, n2);
            const int c = (ti_ + 1) * W1 + (tj_ + 1);
            const int cu = ti_ * WU + tj_;
            const float *u0 = sU[k & 1], *u1 = sU[(k + 1) & 1];
            const float du_v = mv * (u0[cu + WU] - u0[cu]), du_h = mh * (u0[cu + 1] - u0[cu]);
            const float dn_v = mv * (u1[cu + WU] - u1[cu]), dn_h = mh * (u1[cu + 1] - u1[cu]);
            const int64_t q = vox(d, k, i, j);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const float(*W)[S1] = sW[f];
                const float pv = mv * (W[0][c] + 0.25f * ((W[2][c] + W[2][c + W1]) + (W[2][c - 1] + W[2][c + W1 - 1]))
                                       + 0.5f * (W[4][c] + W[4][c + W1]));
                const float ph = mh * (W[3][c] + 0.25f * ((W[1][c] + W[1][c + 1]) + (W[1][c - W1] + W[1][c - W1 + 1]))
                                       + 0.5f * (W[5][c] + W[5][c + 1]));
                const DT *ys = f ? src.y2 : src.y1;
                DT *yd = f ? dst.y2 : dst.y1;
                const float gv = f ? msk * (dn_v - du_v) : du_v;
                const float gh = f ? msk * (dn_h - du_h) : du_h;
                st(yd + q, ld(ys + q) + kStepY * (gv - pv));
                st(yd + N + q, ld(ys + N + q) + kStepY * (gh - ph));
            }
        }
    };

    // prologue: bands kb-1 (for D_s^T at kb) and kb, then u' of band kb
    if (kb >= 1) loadY(kb - 1, (kb - 1) & 1);
    loadY(kb, kb & 1);
    __syncthreads();
    uphase(kb, true);
    __syncthreads();
    for (int k = kb; k < ke; ++k) {
        loadY(k + 1, (k + 1) & 1);  // zeros beyond the last band
        __syncthreads();
        uphase(k + 1, k + 1 < ke);
        wphase(k);
        __syncthreads();
        yphase(k);
        __syncthreads();
    }
    du2 = block_sum<NT>(du2, red);
    u2 = block_sum<NT>(u2, red);
    if (tid == 0) {
        a.part[2 * blockIdx.x] = du2;
        a.part[2 * blockIdx.x + 1] = u2;
    }
}

__device__ __forceinline__ float soft(float z, double tau)
{
    const double m = fabs((double)z) - tau;
    return m > 0.0 ? copysignf((float)m, z) : 0.0f;
}

// Steps 2, 3 (soft thresholds at the selected levels), 7, 8, 13 and 14.
template <typename DT>
__global__ __launch_bounds__(NT) void k_sweep_b(IterArgs<DT> a)
{
    const DevScalars *sc = a.sc;
    if (sc->stop) return;
    __shared__ double red[NT / 64];
    const Dims d = a.d;
    const int par = (int)(sc->iter & 1u);
    const Side<DT> src = a.side[par], dst = a.side[par ^ 1];
    const double ts = sc->sel[0].tau, tt = sc->sel[1].tau;
    const int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x;
    double r2 = 0.0;
    if (q < d.plane) {
        const int i = (int)((q / d.n2) % d.n1);
        const float sn = soft(a.zs[q], ts), tn = soft(a.zt[q], tt);
        const float sp = 2.f * sn - src.s[q], tp = 2.f * tn - src.t[q];
        float tp1 = 0.f;
        if (i <= d.n1 - 2) tp1 = 2.f * soft(a.zt[q + d.n2], tt) - src.t[q + d.n2];
        dst.s[q] = sn;
        dst.t[q] = tn;
        st(dst.y3 + q, ld(src.y3 + q) + kStepY * mask_le(i, d.n1) * (tp1 - tp));
        st(dst.y4 + q, ld(a.y4p + q) + kStepY * (sp + tp));
        const double e = 5.0 * (double)ld(dst.y4 + q) - (double)a.v[q];
        r2 = e * e;
    }
    r2 = block_sum<NT>(r2, red);
    if (threadIdx.x == 0) a.part[2 * a.blocks_a + blockIdx.x] = r2;
}

// Fixed-order sums of the partials; l2-ball factor, stopping rule, counter.
__global__ __launch_bounds__(NT) void k_finalize(DevScalars *sc, const double *part, int blocks_a,
                                                 int blocks_b)
{
    if (sc->stop) return;
    __shared__ double red[NT / 64];
    double du2 = 0.0, u2 = 0.0, r2 = 0.0;
    for (int b = threadIdx.x; b < blocks_a; b += NT) {
        du2 += part[2 * b];
        u2 += part[2 * b + 1];
    }
    for (int b = threadIdx.x; b < blocks_b; b += NT) r2 += part[2 * blocks_a + b];
    du2 = block_sum<NT>(du2, red);
    u2 = block_sum<NT>(u2, red);
    r2 = block_sum<NT>(r2, red);
    if (threadIdx.x == 0) {
        const double r = sqrt(r2);
        const double rel = u2 > 0.0 ? sqrt(du2) / sqrt(u2) : __longlong_as_double(0x7ff0000000000000ll);
        const bool bad = !isfinite(du2) || !isfinite(u2) || !isfinite(r2);
        sc->r = r;
        sc->rel = rel;
        sc->c4 = r > sc->eps ? 1.0 - sc->eps / r : 0.0;
        sc->d4 = 1.0;
        sc->iter = sc->iter + 1u;
        sc->calls_iter = sc->calls_iter + 1u;
        if (bad) sc->nonfinite = 1u;
        if (bad || (sc->tol > 0.0 && rel < sc->tol)) sc->stop = 1u;
    }
}

template <typename DT>
__global__ __launch_bounds__(NT) void k_init(Dims d, const float *v, Side<DT> s0, DevScalars *sc,
                                             double eps, double tol)
{
    const int64_t N = d.plane;
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < N; q += stride) {
        s0.u[q] = v[q];
        s0.s[q] = 0.f;
        s0.t[q] = 0.f;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            s0.w1[c * N + q] = 0.f;
            s0.w2[c * N + q] = 0.f;
        }
        st(s0.y1 + q, 0.f);
        st(s0.y1 + N + q, 0.f);
        st(s0.y2 + q, 0.f);
        st(s0.y2 + N + q, 0.f);
        st(s0.y3 + q, 0.f);
        st(s0.y4 + q, 0.f);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevScalars z = {};
        z.c4 = 1.0;
        z.d4 = 0.0;
        z.eps = eps;
        z.tol = tol;
        *sc = z;
    }
}

__global__ void k_begin_call(DevScalars *sc, double tol)
{
    if (threadIdx.x == 0) {
        sc->tol = tol;
        sc->calls_iter = 0u;
        sc->fallback = 0u;
        if (!sc->nonfinite) sc->stop = 0u;
    }
}

// State copy in/out. var: GEO_VAR_*; planes: 1, 6 or 2.
template <typename DT>
__global__ __launch_bounds__(NT) void k_state_io(Dims d, Side<DT> s0, Side<DT> s1, DevScalars *sc,
                                                 int var, const float *v, float *out,
                                                 const float *in)
{
    const int64_t N = d.plane;
    const int par = (int)(sc->iter & 1u);
    const Side<DT> s = par ? s1 : s0;
    const int planes = (var == GEO_VAR_W1 || var == GEO_VAR_W2) ? 6
                       : (var == GEO_VAR_Y1 || var == GEO_VAR_Y2) ? 2 : 1;
    const int64_t total = N * planes;
    const int64_t stride = (int64_t)gridDim.x * NT;
    const float c4 = (float)sc->c4, d4v = (float)(sc->d4 * 0.2);
    for (int64_t g = (int64_t)blockIdx.x * NT + threadIdx.x; g < total; g += stride) {
        if (out) {
            float x = 0.f;
            switch (var) {
            case GEO_VAR_U: x = s.u[g]; break;
            case GEO_VAR_S: x = s.s[g]; break;
            case GEO_VAR_T: x = s.t[g]; break;
            case GEO_VAR_W1: x = s.w1[g]; break;
            case GEO_VAR_W2: x = s.w2[g]; break;
            case GEO_VAR_Y1: x = ld(s.y1 + g); break;
            case GEO_VAR_Y2: x = ld(s.y2 + g); break;
            case GEO_VAR_Y3: x = ld(s.y3 + g); break;
            default: x = c4 * (ld(s.y4 + g) - d4v * v[g]); break;
            }
            out[g] = x;
        } else {
            const float x = in[g];
            switch (var) {
            case GEO_VAR_U: s.u[g] = x; break;
            case GEO_VAR_S: s.s[g] = x; break;
            case GEO_VAR_T: s.t[g] = x; break;
            case GEO_VAR_W1: s.w1[g] = x; break;
            case GEO_VAR_W2: s.w2[g] = x; break;
            case GEO_VAR_Y1: st(s.y1 + g, x); break;
            case GEO_VAR_Y2: st(s.y2 + g, x); break;
            case GEO_VAR_Y3: st(s.y3 + g, x); break;
            default: st(s.y4 + g, x); break;
            }
        }
    }
}

// y4 loaded as-is: switch its lazy form to y4 = 1 * (stored - 0 * v/5).
__global__ void k_y4_identity(DevScalars *sc)
{
    if (threadIdx.x == 0) {
        sc->c4 = 1.0;
        sc->d4 = 0.0;
    }
}

template <typename DT>
Side<DT> side_of(void *ws, const Layout &L, int p)
{
    char *b = (char *)ws;
    Side<DT> s;
    s.u = (float *)(b + L.u[p]);
    s.s = (float *)(b + L.s[p]);
    s.t = (float *)(b + L.t[p]);
    s.w1 = (float *)(b + L.w1[p]);
    s.w2 = (float *)(b + L.w2[p]);
    s.y1 = (DT *)(b + L.y1[p]);
    s.y2 = (DT *)(b + L.y2[p]);
    s.y3 = (DT *)(b + L.y3[p]);
    s.y4 = (DT *)(b + L.y4[p]);
    return s;
}

int grid_for(int64_t n)
{
    int64_t b = (n + NT - 1) / NT;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

template <typename DT>
IterArgs<DT> iter_args(const Dims &d, const float *v, void *ws, const Layout &L, double omega,
                       double mu_lo, double mu_hi)
{
    char *b = (char *)ws;
    IterArgs<DT> a;
    a.d = d;
    a.v = v;
    a.side[0] = side_of<DT>(ws, L, 0);
    a.side[1] = side_of<DT>(ws, L, 1);
    a.y4p = (DT *)(b + L.y4p);
    a.zs = (float *)(b + L.zs);
    a.zt = (float *)(b + L.zt);
    a.sc = (DevScalars *)(b + L.scalars);
    a.part = (double *)(b + L.partials);
    a.g = sweep_grid(d.n1, d.n2, d.n3);
    a.blocks_a = a.g.blocks();
    a.thr1 = (float)(omega * 0.25);
    a.mu_lo = (float)mu_lo;
    a.mu_hi = (float)mu_hi;
    return a;
}

template <typename DT>
hipError_t iteration_t(const Dims &d, const float *v, void *ws, const Layout &L, const IterParams &ip,
                       hipStream_t st, hipEvent_t *ev)
{
    IterArgs<DT> a = iter_args<DT>(d, v, ws, L, ip.omega, ip.mu_lo, ip.mu_hi);
    Hist *hist = (Hist *)((char *)ws + L.hist);
    const uint32_t *stop = &a.sc->stop;
    const int blocks_b = point_blocks(d.plane);
    if (ev) (void)hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(k_sweep_a<DT>, dim3(a.blocks_a), dim3(NT), 0, st, a);
    if (ev) (void)hipEventRecord(ev[1], st);
    hipError_t e = select_begin(a.sc->sel, 2, ip.alpha, ip.beta, hist, stop, st);
    if (e != hipSuccess) return e;
    e = select_run(a.zs, a.zt, 2, d.plane, a.sc->sel, hist, stop, st);
    if (e != hipSuccess) return e;
    if (ev) (void)hipEventRecord(ev[2], st);
    hipLaunchKernelGGL(k_sweep_b<DT>, dim3(blocks_b), dim3(NT), 0, st, a);
    if (ev) (void)hipEventRecord(ev[3], st);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(NT), 0, st, a.sc, (const double *)a.part,
                       a.blocks_a, blocks_b);
    if (ev) (void)hipEventRecord(ev[4], st);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_iteration(const Dims &d, const float *v, void *ws, const Layout &L,
                            const IterParams &ip, hipStream_t st, hipEvent_t *ev)
{
    return L.dual_bytes == 2 ? iteration_t<bf16>(d, v, ws, L, ip, st, ev)
                             : iteration_t<float>(d, v, ws, L, ip, st, ev);
}

hipError_t launch_init(const Dims &d, const float *v, void *ws, const Layout &L, double eps,
                       double tol, hipStream_t st)
{
    DevScalars *sc = (DevScalars *)((char *)ws + L.scalars);
    if (L.dual_bytes == 2)
        hipLaunchKernelGGL(k_init<bf16>, dim3(grid_for(d.plane)), dim3(NT), 0, st, d, v,
                           side_of<bf16>(ws, L, 0), sc, eps, tol);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(grid_for(d.plane)), dim3(NT), 0, st, d, v,
                           side_of<float>(ws, L, 0), sc, eps, tol);
    return hipGetLastError();
}

hipError_t launch_begin_call(void *ws, const Layout &L, double tol, hipStream_t st)
{
    DevScalars *sc = (DevScalars *)((char *)ws + L.scalars);
    hipLaunchKernelGGL(k_begin_call, dim3(1), dim3(64), 0, st, sc, tol);
    return hipGetLastError();
}

hipError_t launch_state_io(const Dims &d, void *ws, const Layout &L, int var, const float *v,
                           float *out, const float *in, hipStream_t st)
{
    DevScalars *sc = (DevScalars *)((char *)ws + L.scalars);
    const int planes = (var == GEO_VAR_W1 || var == GEO_VAR_W2) ? 6
                       : (var == GEO_VAR_Y1 || var == GEO_VAR_Y2) ? 2 : 1;
    const int grid = grid_for(d.plane * planes);
    if (L.dual_bytes == 2)
        hipLaunchKernelGGL(k_state_io<bf16>, dim3(grid), dim3(NT), 0, st, d, side_of<bf16>(ws, L, 0),
                           side_of<bf16>(ws, L, 1), sc, var, v, out, in);
    else
        hipLaunchKernelGGL(k_state_io<float>, dim3(grid), dim3(NT), 0, st, d,
                           side_of<float>(ws, L, 0), side_of<float>(ws, L, 1), sc, var, v, out, in);
    if (in && var == GEO_VAR_Y4) hipLaunchKernelGGL(k_y4_identity, dim3(1), dim3(64), 0, st, sc);
    return hipGetLastError();
}

}  // namespace geo
