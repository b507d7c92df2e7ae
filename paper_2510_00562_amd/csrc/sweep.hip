// One iteration of Alg. 1 (problem (20)) as HBM-streaming sweeps for gfx950.
//
//   sweep A  (fused, LDS-tiled): steps 1, 4, 5, the extrapolations 6 and 9-10,
//            steps 11 and 12 and the u' part of step 14; it also evaluates the
//            inputs z_s, z_t of the two l1-ball projections (steps 2, 3) and
//            feeds the threshold search (count and sum above a predicted
//            window, values inside it), plus the FP64 partial sums of the
//            stopping rule (eq. (28)).
//   search   (select.hip, fallback.hip): exact soft-threshold levels tau_s,
//            tau_t from the window candidates, or, for a window that
//            missed, from three histogram passes in the same slot.
//   sweep B  (pointwise): steps 2, 3, 7, 8, 13, the rest of step 14 and the
//            FP64 partial sums of the l2-ball distance of step 15.
//   finalize (one block): the l2-ball factor of step 15 (applied lazily when
//            y4 is next read), the stopping test and the iteration counter.
//
// Sweep A keeps the w1/w2 extrapolations (12 of the 21 state words per voxel)
// out of HBM: a workgroup owns a TI x TJ pixel tile and marches through a
// chunk of bands. Per band it stages the masked dual edge fields y1, y2 with
// a 2-pixel halo in LDS, recomputes w' on a 1-pixel ring and u' on the
// (i+1, j+1) ring, and updates y1, y2 from LDS; the D_s coupling of
// neighbouring bands is carried in LDS. Global loads of band k+1 (w) and
// k+2 (y, u, v, y4, s, t, y3) are issued while band k is computed, so the
// memory latency overlaps the arithmetic.
//
// Every state array is ping-ponged: iteration k reads side (k & 1) and writes
// side ((k + 1) & 1), so halo reads never race with writes. The side comes
// from the device iteration counter, which makes one iteration's launches a
// fixed sequence; once the stopping rule holds a device flag turns the
// remaining launches into no-ops, so iteration counts stay exact.
#include <string.h>

#include "radix.hpp"

namespace geo {

namespace {

constexpr int NT = kSweepThreads;
// Tile geometry of shape S (kShapeTI[S] x kShapeTJ[S] pixels)
template <int S>
struct TileOf {
    static constexpr int TI = kShapeTI[S], TJ = kShapeTJ[S];
    static constexpr int H2 = TI + 4, W2 = TJ + 4, S2 = H2 * W2;  // y with a 2-pixel halo
    static constexpr int H1 = TI + 2, W1 = TJ + 2, S1 = H1 * W1;  // w' on a 1-pixel ring
    static constexpr int HU = TI + 1, WU = TJ + 1, SU = HU * WU;  // u' with the (+1, +1) ring
    static constexpr int NY = (S2 + NT - 1) / NT;                  // y points per thread
    static constexpr int RING1 = S1 - TI * TJ;                     // w' ring points
    static constexpr int RINGU = SU - TI * TJ;                     // u' ring points
    static_assert(TI * TJ == NT && TJ % 64 == 0, "one own point per thread, whole wavefronts per tile row");
    static_assert(RING1 <= NT && RINGU <= NT, "at most one ring point per thread");
};
// the geometry of shape S under its short names, inside a kernel
#define GEO_TILE_GEOMETRY(S)                                                              \
    constexpr int TI = TileOf<S>::TI, TJ = TileOf<S>::TJ;                                 \
    constexpr int H2 = TileOf<S>::H2, W2 = TileOf<S>::W2, S2 = TileOf<S>::S2;             \
    constexpr int H1 = TileOf<S>::H1, W1 = TileOf<S>::W1, S1 = TileOf<S>::S1;             \
    constexpr int HU = TileOf<S>::HU, WU = TileOf<S>::WU, SU = TileOf<S>::SU;             \
    constexpr int NY = TileOf<S>::NY, RING1 = TileOf<S>::RING1, RINGU = TileOf<S>::RINGU; \
    (void)H2; (void)W2; (void)S2; (void)H1; (void)W1; (void)S1;                          \
    (void)HU; (void)WU; (void)SU; (void)NY; (void)RING1; (void)RINGU
constexpr int NPT = 256;  // threads of the pointwise kernels

template <typename DT>
using Table = const CubeArgs<DT> *__restrict__;

// Value as stored (FP32 or rounded to BF16), for the l2-ball distance.
__device__ __forceinline__ float as_stored(const float *, float x) { return x; }
__device__ __forceinline__ float as_stored(const bf16 *, float x)
{
    bf16 b;
    st(&b, x);
    return ld(&b);
}

// XCD-aware persistent tile order: the 8 XCDs take contiguous tile ranges so
// that the halos shared by neighbouring tiles meet in the same L2.
__device__ __forceinline__ int tile_at(int b, int G, int T, int r)
{
    if (G >= 8 && (G & 7) == 0) {
        const int x = b & 7, slot = b >> 3, per = G >> 3;
        const int lo = (int)(((int64_t)x * T) >> 3), hi = (int)(((int64_t)(x + 1) * T) >> 3);
        const int t = lo + slot + r * per;
        return t < hi ? t : -1;
    }
    const int t = b + r * G;
    return t < T ? t : -1;
}

// Sums of 8 FP64 values over the block; result valid in thread 0.
__device__ __forceinline__ void block_sum8(double (&x)[8], double *red /* 8 * NT/64 */)
{
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = wave_sum(x[q]);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 8; ++q) red[q * (NT / 64) + wid] = x[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            double t = 0.0;
            for (int w = 0; w < NT / 64; ++w) t += red[q * (NT / 64) + w];
            x[q] = t;
        }
}

template <typename DT, int S>
__global__ __launch_bounds__(NT, 4) void k_sweep_a(Table<DT> cubes, LaunchShape sh)
{
    GEO_TILE_GEOMETRY(S);
    using P = typename PairOf<DT>::type;
    // [band parity][y1v, y1h, y2v, y2h] masked | u' by band parity |
    // w1', w2' planes read by neighbours (ud_h, lr_v, c_v, c_h)
    __shared__ __align__(16) float smem[2 * 4 * S2 + 2 * SU + 2 * 4 * S1];
    float(*sY)[4][S2] = reinterpret_cast<float(*)[4][S2]>(smem);
    float(*sU)[SU] = reinterpret_cast<float(*)[SU]>(smem + 2 * 4 * S2);
    float(*sW)[4][S1] = reinterpret_cast<float(*)[4][S1]>(smem + 2 * 4 * S2 + 2 * SU);
    __shared__ double red[8 * (NT / 64)];
    __shared__ uint32_t ncand[2];
    __shared__ int tile0[kMaxBatch + 1];

    // The tiles of the cubes of this tile shape that work in this slot, one
    // cube after another: a cube that idles takes none, so the persistent
    // blocks, and the XCDs, share the working cubes' tiles evenly (with the
    // full list, a batch in which a few cubes still run would leave most
    // blocks without work). Every block reads the same flags, written before
    // this launch.
    static_assert(kMaxBatch <= 64, "one wavefront scans the cubes");
    if (threadIdx.x < 64) {
        const int c = threadIdx.x;
        int x = c < sh.ncubes && cubes[c].c.g.shape == S && !idle(cubes[c].c.sc) ? cubes[c].c.ntiles : 0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (c >= o) x += y;
        }
        if (c < sh.ncubes) tile0[c + 1] = x;
        if (c == 0) tile0[0] = 0;
    }
    __syncthreads();
    const int tid = threadIdx.x;
    const int oti = tid / TJ, otj = tid % TJ;  // the thread's own point in the tile

    // ring coordinates (R1-local for w', RU-local for u')
    int rwi = 0, rwj = 0, rui = 0, ruj = 0;
    if (tid < RING1) {
        if (tid < W1) { rwi = 0; rwj = tid; }
        else if (tid < 2 * W1) { rwi = H1 - 1; rwj = tid - W1; }
        else { const int s = tid - 2 * W1; rwi = 1 + (s >> 1); rwj = (s & 1) ? W1 - 1 : 0; }
    }
    if (tid < RINGU) {
        if (tid < WU) { rui = TI; ruj = tid; }
        else { rui = tid - WU; ruj = TJ; }
    }
    const bool ring_w = tid < RING1, ring_u = tid < RINGU;

    for (int r = 0;; ++r) {
        // (the working cubes' tile count is read from LDS at each tile rather
        // than kept live through the march)
        const int t = tile_at(blockIdx.x, sh.shape_grid[S], tile0[sh.ncubes], r);
        if (t < 0) break;
        int cube = 0;
        while (tile0[cube + 1] <= t) ++cube;
        // uniform across the block: the cube's entry is read with scalar loads
        cube = __builtin_amdgcn_readfirstlane(cube);
        const int lt = __builtin_amdgcn_readfirstlane(t - tile0[cube]);  // tile within the cube
        const4<CubeArgs<DT>> &a = ((const4<CubeArgs<DT>> *)cubes)[cube];
        DevScalars *sc = a.c.sc;
        // Never taken (an idle cube has no tiles in the list); without it the
        // register allocation of one of the sweep's forms spills.
        if (idle(sc)) continue;
        const SweepGrid g{a.c.g.tj, a.c.g.ti, a.c.g.tk, a.c.g.kc, S};
        const int tj = lt % g.tj, rest = lt / g.tj;
        const int j0 = tj * TJ, i0 = (rest % g.ti) * TI, kb = (rest / g.ti) * g.kc;
        const Dims d = load_dims(a.c.d);
        const int n1 = d.n1, n2 = d.n2, n3 = d.n3;
        const int ke = min(kb + g.kc, n3);

        const uint32_t N = (uint32_t)d.plane;
        if (tid < 2) ncand[tid] = 0u;  // published by the first barrier of the march
        const int par = (int)(sc->iter & 1u);
        const Side<DT> src = load_side(a.side[par]), dst = load_side(a.side[par ^ 1]);
        const float a4 = (float)sc->a4;
        auto vox32 = [&](int k, int i, int j) {
            return ((uint32_t)k * (uint32_t)n1 + (uint32_t)i) * (uint32_t)n2 + (uint32_t)j;
        };
        const bool zst = sc->zstore != 0u;
        float wlo[2], whi[2];
        bool won[2];
        for (int f = 0; f < 2; ++f) {
            won[f] = sc->sel[f].win_on != 0u;
            wlo[f] = sc->sel[f].win_lo;
            whi[f] = sc->sel[f].win_hi;
        }
        double du2 = 0.0, u2 = 0.0;
        double s_hi[2] = {0.0, 0.0}, s_all[2] = {0.0, 0.0};
        float c_hi[2] = {0.f, 0.f};
        const int oi = i0 + oti, oj = j0 + otj;
        const bool own_in = oi < n1 && oj < n2;

        // ---------------- register staging of global loads ----------------
        float2 ry1[NY], ry2[NY];
        auto loadY = [&](int k) {
#pragma unroll
            for (int n = 0; n < NY; ++n) {
                const int p = tid + NT * n;
                const int li = p / W2, lj = p - li * W2;
                const int i = i0 - 2 + li, j = j0 - 2 + lj;
                float2 y1 = make_float2(0.f, 0.f), y2 = y1;
                if (p < S2 && k >= 0 && k < n3 && i >= 0 && i < n1 && j >= 0 && j < n2) {
                    const uint32_t q = vox32(k, i, j);
                    y1 = ld2(src.y1 + q);
                    y2 = ld2(src.y2 + q);
                    if (i > n1 - 2) y1.x = y2.x = 0.f;  // masked: last row (vertical)
                    if (j > n2 - 2) y1.y = y2.y = 0.f;  // masked: last column (horizontal)
                }
                ry1[n] = y1;
                ry2[n] = y2;
            }
        };
        auto storeY = [&](int buf) {
#pragma unroll
            for (int n = 0; n < NY; ++n) {
                const int p = tid + NT * n;
                if (p < S2) {
                    sY[buf][0][p] = ry1[n].x;
                    sY[buf][1][p] = ry1[n].y;
                    sY[buf][2][p] = ry2[n].x;
                    sY[buf][3][p] = ry2[n].y;
                }
            }
        };
        // u, y4 (stored) at the own point and the u' ring point; v, s, t,
        // y3 (row and row above) at the own point
        float ru_u, ru_y4, ru_v, ru_s, ru_t, ru_y3c, ru_y3m, rr_u, rr_y4;
        auto loadRU = [&](int kk) {
            ru_u = ru_y4 = ru_v = ru_s = ru_t = ru_y3c = ru_y3m = 0.f;
            if (kk < n3 && own_in) {
                const uint32_t q = vox32(kk, oi, oj);
                ru_u = src.u[q];
                ru_y4 = ld(src.y4 + q);
                ru_v = ld_nt(a.c.v + q);
                ru_s = ld_nt(src.s + q);
                ru_t = ld_nt(src.t + q);
                ru_y3c = oi <= n1 - 2 ? ld(src.y3 + q) : 0.f;
                ru_y3m = oi >= 1 ? ld(src.y3 + q - n2) : 0.f;
            }
            rr_u = rr_y4 = 0.f;
            const int i = i0 + rui, j = j0 + ruj;
            if (ring_u && kk < n3 && i < n1 && j < n2) {
                const uint32_t q = vox32(kk, i, j);
                rr_u = src.u[q];
                rr_y4 = ld(src.y4 + q);
            }
        };
        // w1, w2 (3 pairs each) at the own point and the w' ring point
        float2 rw[2][2][3];  // [own, ring][field][grid]
        auto loadW = [&](int k) {
#pragma unroll
            for (int o = 0; o < 2; ++o) {
                const int i = o == 0 ? oi : i0 - 1 + rwi, j = o == 0 ? oj : j0 - 1 + rwj;
                const bool in = (o == 0 ? true : ring_w) && i >= 0 && i < n1 && j >= 0 && j < n2 && k < n3;
                const uint32_t q = in ? vox32(k, i, j) : 0u;
#pragma unroll
                for (int f = 0; f < 2; ++f) {
                    const float2 *w = f ? src.w2 : src.w1;
                    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
                    float2 c = make_float2(0.f, 0.f);
                    if (in) {
                        a = w_udlr(w)[q];
                        c = w_c(w, N)[q];
                    }
                    rw[o][f][0] = make_float2(a.x, a.y);
                    rw[o][f][1] = make_float2(a.z, a.w);
                    rw[o][f][2] = c;
                }
            }
        };

        // ---------------- phases ----------------
        auto dT = [&](int buf, int pv, int c) {
            const float *yv = sY[buf][pv], *yh = sY[buf][pv + 1];
            return (yv[c - W2] - yv[c]) + (yh[c - 1] - yh[c]);
        };
        // u+ of step 1 and u' at one point of band kk
        auto u_at = [&](int kk, int ui, int uj, float uo, float y4s, float &y4) {
            const int buf = kk & 1;
            const int c = (ui + 2) * W2 + (uj + 2);
            float g = dT(buf, 0, c);                  // D^T y1
            if (kk <= n3 - 2) g -= dT(buf, 2, c);      // D_s^T D^T y2
            if (kk >= 1) g += dT(buf ^ 1, 2, c);
            y4 = y4_of(y4s, a4);
            const float x = uo - kStepU * (g + y4);
            return x < a.c.mu_lo ? a.c.mu_lo : (x > a.c.mu_hi ? a.c.mu_hi : x);
        };
        // step 1 (u+), u' and the z inputs of steps 2, 3 for band kk
        auto uphase = [&](int kk, bool own_band) {
            const int buf = kk & 1;
            float up = 0.f, zs = 0.f, zt = 0.f;
            bool wr = false;
            if (kk < n3 && own_in) {
                float y4;
                const float un = u_at(kk, oti, otj, ru_u, ru_y4, y4);
                up = 2.f * un - ru_u;
                if (own_band) {
                    wr = true;
                    const uint32_t q = vox32(kk, oi, oj);
                    st_nt(dst.u + q, un);
                    // 5 (y4 + u'/5) - v: step 14 without s', t', times 5, minus v
                    st_nt(a.y4p + q, (5.f * y4 + up) - ru_v);
                    const double dl = (double)un - (double)ru_u;
                    du2 += dl * dl;
                    u2 += (double)ru_u * (double)ru_u;
                    zs = zs_of(ru_s, y4);
                    zt = zt_of(ru_t, ru_y3m, ru_y3c, y4);
                    if (zst) {
                        a.c.zbuf[q] = zs;
                        a.c.zbuf[N + q] = zt;
                    }
                }
            }
            sU[buf][oti * WU + otj] = up;
            if (ring_u) {
                float upr = 0.f;
                if (kk < n3 && i0 + rui < n1 && j0 + ruj < n2) {
                    float y4;
                    const float un = u_at(kk, rui, ruj, rr_u, rr_y4, y4);
                    upr = 2.f * un - rr_u;
                }
                sU[buf][rui * WU + ruj] = upr;
            }
            // threshold-search inputs (every lane takes part)
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const float av = fabsf(f ? zt : zs);
                bool cand = false;
                if (wr) {
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
                wave_append(cand, av, a.c.cand + ((int64_t)f * a.c.ntiles + lt) * a.c.capt,
                            &ncand[f], a.c.capt);
            }
        };
        // steps 4, 5 and the w extrapolations (9, 10) at one point of band k;
        // own: also writes w+ and returns the own-only planes ud_v', lr_h'
        float wk[2][2];
        auto w_at = [&](int k, int o, int wi, int wj, bool act) {
            const int buf = k & 1;
            const int i = i0 - 1 + wi, j = j0 - 1 + wj;
            const bool in = act && i >= 0 && i < n1 && j >= 0 && j < n2;
            const float mv = mask_le(i, n1), mh = mask_le(j, n2);
            const int c = (wi + 1) * W2 + (wj + 1), c1 = wi * W1 + wj;
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                float o6[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                if (in) {
                    const float *yv = sY[buf][2 * f], *yh = sY[buf][2 * f + 1];
                    float L[6];
                    L[0] = mv * yv[c];
                    L[1] = mv * 0.25f * ((yh[c] + yh[c - 1]) + (yh[c + W2] + yh[c + W2 - 1]));
                    L[2] = mh * 0.25f * ((yv[c] + yv[c - W2]) + (yv[c + 1] + yv[c - W2 + 1]));
                    L[3] = mh * yh[c];
                    L[4] = 0.5f * (yv[c] + yv[c - W2]);
                    L[5] = 0.5f * (yh[c] + yh[c - 1]);
                    const float thr = f ? kStepW : a.c.thr1;
                    float wo[6], wn[6];
#pragma unroll
                    for (int g = 0; g < 3; ++g) {
                        wo[2 * g] = rw[o][f][g].x;
                        wo[2 * g + 1] = rw[o][f][g].y;
                    }
#pragma unroll
                    for (int cc = 0; cc < 6; ++cc) wn[cc] = wo[cc] + kStepW * L[cc];
                    shrink2(wn[0], wn[1], thr);
                    shrink2(wn[2], wn[3], thr);
                    shrink2(wn[4], wn[5], thr);
                    if (o == 0) {
                        const uint32_t q = vox32(k, i, j);
                        float2 *wd = f ? dst.w2 : dst.w1;
                        st_nt(w_udlr(wd) + q, make_float4(wn[0], wn[1], wn[2], wn[3]));
                        st_nt(w_c(wd, N) + q, make_float2(wn[4], wn[5]));
                    }
#pragma unroll
                    for (int cc = 0; cc < 6; ++cc) o6[cc] = 2.f * wn[cc] - wo[cc];
                    o6[0] *= mv;
                    o6[1] *= mv;
                    o6[2] *= mh;
                    o6[3] *= mh;
                }
                if (act) {
                    sW[f][0][c1] = o6[1];
                    sW[f][1][c1] = o6[2];
                    sW[f][2][c1] = o6[4];
                    sW[f][3][c1] = o6[5];
                }
                if (o == 0) {
                    wk[f][0] = o6[0];
                    wk[f][1] = o6[3];
                }
            }
        };
        auto wphase = [&](int k) {
            w_at(k, 0, oti + 1, otj + 1, true);
            if (ring_w) w_at(k, 1, rwi, rwj, true);
        };
        // steps 11, 12 for band k at the own point
        auto yphase = [&](int k) {
            if (!own_in) return;
            const float msk = k <= n3 - 2 ? 1.f : 0.f;
            const int buf = k & 1;
            const float mv = mask_le(oi, n1), mh = mask_le(oj, n2);
            const int c1 = (oti + 1) * W1 + (otj + 1);
            const int c2 = (oti + 2) * W2 + (otj + 2);
            const int cu = oti * WU + otj;
            const float *u0 = sU[buf], *u1 = sU[buf ^ 1];
            const float du_v = mv * (u0[cu + WU] - u0[cu]), du_h = mh * (u0[cu + 1] - u0[cu]);
            const float dn_v = mv * (u1[cu + WU] - u1[cu]), dn_h = mh * (u1[cu + 1] - u1[cu]);
            const uint32_t q = vox32(k, oi, oj);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const float(*W)[S1] = sW[f];
                const float pv = mv * (wk[f][0] + 0.25f * ((W[1][c1] + W[1][c1 + W1]) + (W[1][c1 - 1] + W[1][c1 + W1 - 1]))
                                       + 0.5f * (W[2][c1] + W[2][c1 + W1]));
                const float ph = mh * (wk[f][1] + 0.25f * ((W[0][c1] + W[0][c1 + 1]) + (W[0][c1 - W1] + W[0][c1 - W1 + 1]))
                                       + 0.5f * (W[3][c1] + W[3][c1 + 1]));
                P *yd = f ? dst.y2 : dst.y1;
                const float2 y = make_float2(sY[buf][2 * f][c2], sY[buf][2 * f + 1][c2]);
                const float gv = f ? msk * (dn_v - du_v) : du_v;
                const float gh = f ? msk * (dn_h - du_h) : du_h;
                const float2 yn = make_float2(y.x + kStepY * (gv - pv), y.y + kStepY * (gh - ph));
                // A masked entry (vertical component on the last row,
                // horizontal on the last column) keeps its value, and both
                // sides hold the same one: it is not written at all.
                const bool mx = oi > n1 - 2, my = oj > n2 - 2;
                if (!mx && !my) st2_nt(yd + q, yn);
                else if (!mx) st_comp_nt(yd + q, 0, yn.x);
                else if (!my) st_comp_nt(yd + q, 1, yn.y);
            }
        };

        // ---------------- march through the band chunk ----------------
        if (kb >= 1) {
            loadY(kb - 1);
            storeY((kb - 1) & 1);
        }
        loadY(kb);
        loadRU(kb);
        storeY(kb & 1);
        __syncthreads();
        uphase(kb, true);
        loadY(kb + 1);
        loadRU(kb + 1);
        loadW(kb);
        __syncthreads();
        storeY((kb + 1) & 1);
        __syncthreads();
        for (int k = kb; k < ke; ++k) {
            const bool more = k + 1 < ke;
            if (more) loadY(k + 2);
            uphase(k + 1, more);
            if (more) loadRU(k + 2);
            wphase(k);
            if (more) loadW(k + 1);
            __syncthreads();
            yphase(k);
            __syncthreads();
            if (more) storeY(k & 1);
            __syncthreads();
        }

        // the tile's FP64 partials: stopping sums, window statistics
        double acc[8] = {du2, u2, (double)c_hi[0], s_hi[0], s_all[0], (double)c_hi[1], s_hi[1], s_all[1]};
        block_sum8(acc, red);
        if (tid == 0) {
            const int nt = a.c.ntiles;
            a.c.ccount[lt] = ncand[0];
            a.c.ccount[nt + lt] = ncand[1];
            a.c.part[2 * lt] = acc[0];
            a.c.part[2 * lt + 1] = acc[1];
            for (int f = 0; f < 2; ++f)
                for (int q = 0; q < 3; ++q) a.c.winpart[((int64_t)f * nt + lt) * 3 + q] = acc[2 + 3 * f + q];
        }
        __syncthreads();  // red and ncand are reused by the next tile
    }
}

__device__ __forceinline__ float soft(float z, double tau)
{
    const double m = fabs((double)z) - tau;
    return m > 0.0 ? copysignf((float)m, z) : 0.0f;
}

constexpr int RB = kSweepBRows;  // rows per sweep B strip
constexpr int kPrefetchBlocks = 240;  // cache prefetch beside the search
// CPT consecutive values of one row: one 4- or 8-byte access for a pair.
__device__ __forceinline__ void ldv(const float *p, float (&o)[1]) { o[0] = *p; }
__device__ __forceinline__ void ldv(const bf16 *p, float (&o)[1]) { o[0] = ld(p); }
__device__ __forceinline__ void ldv(const float *p, float (&o)[2])
{
    const float2 x = *reinterpret_cast<const float2 *>(p);
    o[0] = x.x;
    o[1] = x.y;
}
__device__ __forceinline__ void ldv(const bf16 *p, float (&o)[2])
{
    const float2 x = ld2(reinterpret_cast<const bf16x2 *>(p));
    o[0] = x.x;
    o[1] = x.y;
}
__device__ __forceinline__ void ldv_nt(const float *p, float (&o)[1]) { o[0] = ld_nt(p); }
__device__ __forceinline__ void ldv_nt(const bf16 *p, float (&o)[1]) { o[0] = ld_nt(p); }
__device__ __forceinline__ void ldv_nt(const float *p, float (&o)[2])
{
    const f32x2 x = __builtin_nontemporal_load(reinterpret_cast<const f32x2 *>(p));
    o[0] = x.x;
    o[1] = x.y;
}
__device__ __forceinline__ void ldv_nt(const bf16 *p, float (&o)[2])
{
    const uint32_t b = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(p));
    o[0] = __uint_as_float(b << 16);
    o[1] = __uint_as_float(b & 0xffff0000u);
}
// four columns: one 16-byte FP32 or 8-byte BF16 access
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void ldv(const float *p, float (&o)[4])
{
    const float4 x = *reinterpret_cast<const float4 *>(p);
    o[0] = x.x;
    o[1] = x.y;
    o[2] = x.z;
    o[3] = x.w;
}
__device__ __forceinline__ void ldv(const bf16 *p, float (&o)[4])
{
    const uint2 b = *reinterpret_cast<const uint2 *>(p);
    o[0] = __uint_as_float(b.x << 16);
    o[1] = __uint_as_float(b.x & 0xffff0000u);
    o[2] = __uint_as_float(b.y << 16);
    o[3] = __uint_as_float(b.y & 0xffff0000u);
}
__device__ __forceinline__ void ldv_nt(const float *p, float (&o)[4])
{
    const f32x4 x = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p));
    o[0] = x.x;
    o[1] = x.y;
    o[2] = x.z;
    o[3] = x.w;
}
__device__ __forceinline__ void ldv_nt(const bf16 *p, float (&o)[4])
{
    float a[2], b[2];
    ldv_nt(p, a);
    ldv_nt(p + 2, b);
    o[0] = a[0];
    o[1] = a[1];
    o[2] = b[0];
    o[3] = b[1];
}
template <typename T>
__device__ __forceinline__ void stv_nt(T *p, const float (&x)[1]) { st_nt(p, x[0]); }
__device__ __forceinline__ void stv_nt(float *p, const float (&x)[4])
{
    f32x4 v;
    v.x = x[0];
    v.y = x[1];
    v.z = x[2];
    v.w = x[3];
    __builtin_nontemporal_store(v, reinterpret_cast<f32x4 *>(p));
}
__device__ __forceinline__ void stv_nt(bf16 *p, const float (&x)[4])
{
    st2_nt(reinterpret_cast<bf16x2 *>(p), make_float2(x[0], x[1]));
    st2_nt(reinterpret_cast<bf16x2 *>(p + 2), make_float2(x[2], x[3]));
}
__device__ __forceinline__ void stv_nt(float *p, const float (&x)[2])
{
    st_nt(reinterpret_cast<float2 *>(p), make_float2(x[0], x[1]));
}
__device__ __forceinline__ void stv_nt(bf16 *p, const float (&x)[2])
{
    st2_nt(reinterpret_cast<bf16x2 *>(p), make_float2(x[0], x[1]));
}

// Steps 2, 3 (soft thresholds at the selected levels), 7, 8, 13 and 14; the
// z inputs are evaluated again exactly as sweep A did. A thread takes a strip
// of RB rows and CPT adjacent columns of one band and issues all of its loads
// at once; only the rows just above and below the strip (D_v coupling of t'
// and y3) are read twice. CPT = 2 (one access per pair) when the row length
// is even, else 1.
template <typename DT, int CPT>
__device__ __forceinline__ double sweep_b_strips(const CubeArgs<DT> &a, const DevScalars *sc, int lb,
                                                 double ts, double tt)
{
    const Dims d = a.c.d;
    const int n1 = d.n1, n2 = d.n2, n3 = d.n3;
    const int par = (int)(sc->iter & 1u);
    const Side<DT> src = a.side[par], dst = a.side[par ^ 1];
    const float a4 = (float)sc->a4;
    double r2 = 0.0;
    const uint32_t nstrip = (uint32_t)((n1 + RB - 1) / RB);
    const uint32_t ncol = (uint32_t)(n2 / CPT);
    const uint32_t items = (uint32_t)n3 * nstrip * ncol;
    const uint32_t stride = (uint32_t)a.c.nb * NPT;
    for (uint32_t w = (uint32_t)lb * NPT + threadIdx.x; w < items; w += stride) {
        const uint32_t j = CPT * (w % ncol), rr = w / ncol;
        const int ia = (int)(rr % nstrip) * RB, k = (int)(rr / nstrip);
        const uint32_t q0 = ((uint32_t)k * (uint32_t)n1 + (uint32_t)ia) * (uint32_t)n2 + j;
        // rows ia .. ia+RB-1 of the strip, and row ia+RB for the D_v coupling
        float y3r[RB + 1][CPT], y4[RB + 1][CPT], to[RB + 1][CPT], so[RB][CPT], yp[RB][CPT];
        float y3m0[CPT];
        if (ia >= 1) ldv(src.y3 + q0 - n2, y3m0);
        else
#pragma unroll
            for (int c = 0; c < CPT; ++c) y3m0[c] = 0.f;
#pragma unroll
        for (int r = 0; r <= RB; ++r) {
            const bool in = ia + r < n1;
            const uint32_t q = q0 + (uint32_t)(r * n2);
            float q4[CPT];
            if (in) {
                ldv(src.y3 + q, y3r[r]);
                ldv(src.y4 + q, q4);
                ldv(src.t + q, to[r]);
                if (r < RB) {
                    ldv_nt(src.s + q, so[r]);
                    ldv_nt(a.y4p + q, yp[r]);
                }
            } else {
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    y3r[r][c] = q4[c] = to[r][c] = 0.f;
                    if (r < RB) so[r][c] = yp[r][c] = 0.f;
                }
            }
#pragma unroll
            for (int c = 0; c < CPT; ++c) y4[r][c] = in ? y4_of(q4[c], a4) : 0.f;
        }
        float tp[RB + 1][CPT];
#pragma unroll
        for (int r = 0; r <= RB; ++r) {
            const int i = ia + r;
            float tn[CPT];
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const float y3m = r == 0 ? y3m0[c] : y3r[r - 1][c];
                tn[c] = soft(zt_of(to[r][c], y3m, i <= n1 - 2 ? y3r[r][c] : 0.f, y4[r][c]), tt);
                tp[r][c] = 2.f * tn[c] - to[r][c];
            }
            if (r < RB && i < n1) stv_nt(dst.t + q0 + (uint32_t)(r * n2), tn);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = ia + r;
            if (i < n1) {
                const uint32_t q = q0 + (uint32_t)(r * n2);
                float sn[CPT], y3n[CPT], qn[CPT];
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    sn[c] = soft(zs_of(so[r][c], y4[r][c]), ts);
                    const float sp = 2.f * sn[c] - so[r][c];
                    const float tp1 = i <= n1 - 2 ? tp[r + 1][c] : 0.f;
                    y3n[c] = y3r[r][c] + kStepY * mask_le(i, n1) * (tp1 - tp[r][c]);
                    // q+ = 5 y4' - v (step 14); r = ||q+|| (step 15)
                    qn[c] = as_stored(dst.y4, yp[r][c] + (sp + tp[r][c]));
                    r2 += (double)qn[c] * (double)qn[c];
                }
                stv_nt(dst.s + q, sn);
                stv_nt(dst.y3 + q, y3n);
                stv_nt(dst.y4 + q, qn);
            }
        }
    }
    return r2;
}

// WIDE: the cubes whose sweep B takes four columns per thread (a kernel of
// their own: that form needs 104 registers, the others 73, and a kernel runs
// at the occupancy of its largest form); otherwise the others.
template <typename DT, bool WIDE>
__global__ __launch_bounds__(NPT) void k_sweep_b(Table<DT> cubes, LaunchShape sh)
{
    __shared__ double red[NPT / 64];
    __shared__ int cube_of_block;
    // blocks [b0, b0 + nb) belong to one cube: the last cube whose b0 is at
    // most this block's index, found by one wavefront (one load per lane;
    // a scan by one thread took a memory round trip per cube of a batch)
    static_assert(kMaxBatch <= 64, "one wavefront covers the cubes");
    if (threadIdx.x < 64) {
        const int c = threadIdx.x;
        const bool le = c < sh.ncubes && cubes[c].c.b0 <= (int)blockIdx.x;
        const unsigned long long m = __ballot(le);
        if (c == 0) cube_of_block = 63 - __clzll((long long)m);  // cube 0 starts at block 0
    }
    __syncthreads();
    const CubeArgs<DT> &a = cubes[__builtin_amdgcn_readfirstlane(cube_of_block)];
    const DevScalars *sc = a.c.sc;
    const int cpt = sweep_b_cpt(a.c.d.n2, (int)sizeof(DT));
    if (idle(sc) || (cpt == 4) != WIDE) return;
    // a missed window's threshold comes from this slot's histogram passes
    const double ts = sc->sel[0].done ? sc->sel[0].tau : fb_final(a.c.rec, 0).tau;
    const double tt = sc->sel[1].done ? sc->sel[1].tau : fb_final(a.c.rec, 1).tau;
    const int lb = (int)blockIdx.x - a.c.b0;  // block within the cube
    double r2;
    if constexpr (WIDE)
        r2 = sweep_b_strips<DT, 4>(a, sc, lb, ts, tt);
    else
        r2 = cpt == 2 ? sweep_b_strips<DT, 2>(a, sc, lb, ts, tt) : sweep_b_strips<DT, 1>(a, sc, lb, ts, tt);
    const double tot = block_sum<NPT>(r2, red);
    if (threadIdx.x == 0) a.c.part[2 * a.c.ntiles + lb] = tot;
}

// Fixed-order sums of the block partials of both sweeps: relative change of u
// (stopping rule), r = ||y4'/gamma4 - v|| for the lazy scale of y4 (step 15),
// iteration counter. A separate one-block launch: a last-block-done pattern
// inside sweep B needs a device-scope release per block, which writes back
// the XCD's L2 each time.
// One block per cube of the table (entries of `stride` bytes).
__global__ __launch_bounds__(NPT) void k_finalize(const char *table, int stride)
{
    // the launch table through the constant address space (scalar loads)
    const4<CubeCommon> &cc = *(const4<CubeCommon> *)(table + (size_t)blockIdx.x * stride);
    DevScalars *sc = cc.sc;
    const double *part = cc.part;
    const int grid_a = cc.ntiles, blocks_b = cc.nb;
    __shared__ double red[3 * (NPT / 64)];
    // the partials are read together with the flag that may make them moot
    const bool skip = idle(sc);
    // each thread adds its partials b = tid, tid + NPT, ... in that order,
    // kFinUnroll of them loaded at a time
    constexpr int kFinUnroll = 8;
    double du2 = 0.0, u2 = 0.0, r2 = 0.0;
    for (int b0 = threadIdx.x; b0 < grid_a; b0 += kFinUnroll * NPT) {
        double x0[kFinUnroll], x1[kFinUnroll];
#pragma unroll
        for (int k = 0; k < kFinUnroll; ++k) {
            const int b = b0 + k * NPT;
            x0[k] = b < grid_a ? part[2 * b] : 0.0;
            x1[k] = b < grid_a ? part[2 * b + 1] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kFinUnroll; ++k)
            if (b0 + k * NPT < grid_a) {
                du2 += x0[k];
                u2 += x1[k];
            }
    }
    for (int b0 = threadIdx.x; b0 < blocks_b; b0 += kFinUnroll * NPT) {
        double x2[kFinUnroll];
#pragma unroll
        for (int k = 0; k < kFinUnroll; ++k) {
            const int b = b0 + k * NPT;
            x2[k] = b < blocks_b ? part[2 * grid_a + b] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kFinUnroll; ++k)
            if (b0 + k * NPT < blocks_b) r2 += x2[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *slot_flags(table, (int)gridDim.x) = 0u;
    if (skip) return;
    // a threshold found by this slot's histogram passes becomes the field's
    // search state, with the window of the next iteration sized by the
    // density of |z| around it (only this block writes the cube's state)
    if (threadIdx.x == 0) {
        bool missed = false;
        for (int f = 0; f < 2; ++f)
            if (!sc->sel[f].done) {
                missed = true;
                const FbRec &r = fb_final(cc.rec, f);
                SelState o = sc->sel[f];
                o.tau = r.tau;
                o.done = 1u;
                o.full = 0u;
                o.dens = cc.rec[f].dens;
                set_window(o, true, window_budget(cc.d.plane));
                sc->sel[f] = o;
            }
        // whether the next iteration's sweep A stores z (iter counts this one)
        const uint32_t calm = missed ? 0u : sc->calm + 1u;
        sc->calm = calm;
        sc->zstore = (sc->iter + 1u < kZStoreIters || calm < kZStoreCalm) ? 1u : 0u;
    }
    // the three block sums at once, in the order of block_sum: a butterfly
    // within each wavefront, then the wavefronts in order (thread 0)
    du2 = wave_sum(du2);
    u2 = wave_sum(u2);
    r2 = wave_sum(r2);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[wid] = du2;
        red[NPT / 64 + wid] = u2;
        red[2 * (NPT / 64) + wid] = r2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        du2 = u2 = r2 = 0.0;
        for (int w = 0; w < NPT / 64; ++w) {
            du2 += red[w];
            u2 += red[NPT / 64 + w];
            r2 += red[2 * (NPT / 64) + w];
        }
        const double r = sqrt(r2);
        const double rel = u2 > 0.0 ? sqrt(du2) / sqrt(u2) : __longlong_as_double(0x7ff0000000000000ll);
        const bool bad = !isfinite(du2) || !isfinite(u2) || !isfinite(r2);
        sc->r = r;
        sc->rel = rel;
        sc->c4 = r > sc->eps ? 1.0 - sc->eps / r : 0.0;
        sc->a4 = sc->gy4 * sc->c4;
        sc->iter = sc->iter + 1u;
        sc->calls_iter = sc->calls_iter + 1u;
        if (bad) sc->nonfinite = 1u;
        // eq. (28), from the second iteration after the initial point on: the
        // first one (zero duals) changes u only by the box projection
        if (bad || (sc->tol > 0.0 && sc->iter >= 2u && rel < sc->tol)) sc->stop = 1u;
    }
}

template <typename DT>
__global__ __launch_bounds__(NPT) void k_init(Dims d, const float *v, Side<DT> s0, Side<DT> s1,
                                              DevScalars *sc, double eps, double tol, double alpha,
                                              double beta)
{
    using P = typename PairOf<DT>::type;
    const int64_t N = d.plane;
    const int64_t stride = (int64_t)gridDim.x * NPT;
    const float2 z2 = make_float2(0.f, 0.f);
    for (int64_t q = (int64_t)blockIdx.x * NPT + threadIdx.x; q < N; q += stride) {
        s0.u[q] = v[q];
        s0.s[q] = 0.f;
        s0.t[q] = 0.f;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            s0.w1[g * N + q] = z2;
            s0.w2[g * N + q] = z2;
        }
        // y1, y2 on both sides: their masked entries are never rewritten
        st2((P *)s0.y1 + q, z2);
        st2((P *)s0.y2 + q, z2);
        st2((P *)s1.y1 + q, z2);
        st2((P *)s1.y2 + q, z2);
        st(s0.y3 + q, 0.f);
        st(s0.y4 + q, 0.f);
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
        z.gy4 = 0.2;  // the y4 step printed after eq. (24)
        *sc = z;
    }
}

__global__ void k_begin_call(DevScalars *sc, double tol, double alpha, double beta, uint32_t limit)
{
    if (threadIdx.x == 0) {
        sc->tol = tol;
        sc->calls_iter = 0u;
        sc->call_limit = limit;
        sc->fallback = 0u;
        sc->sel[0].radius = alpha;
        sc->sel[1].radius = beta;
        if (!sc->nonfinite) sc->stop = 0u;
    }
}

// State copy in/out between separate FP32 planes (the ABI layout) and the
// workspace layout. var: GEO_VAR_*; planes: 1, 6 or 2.
template <typename DT>
__global__ __launch_bounds__(NPT) void k_state_io(Dims d, Side<DT> s0, Side<DT> s1, DevScalars *sc,
                                                  int var, const float *v, float *out,
                                                  const float *in)
{
    using P = typename PairOf<DT>::type;
    const int64_t N = d.plane;
    const int par = (int)(sc->iter & 1u);
    const Side<DT> s = par ? s1 : s0;
    const int planes = (var == GEO_VAR_W1 || var == GEO_VAR_W2) ? 6
                       : (var == GEO_VAR_Y1 || var == GEO_VAR_Y2) ? 2 : 1;
    const int64_t total = N * planes;
    const int64_t stride = (int64_t)gridDim.x * NPT;
    const float a4 = (float)sc->a4;
    for (int64_t g = (int64_t)blockIdx.x * NPT + threadIdx.x; g < total; g += stride) {
        const int pl = (int)(g / N);
        const int64_t q = g - (int64_t)pl * N;
        float2 *wp = var == GEO_VAR_W1 ? s.w1 : s.w2;
        P *yp = var == GEO_VAR_Y1 ? s.y1 : s.y2;
        if (out) {
            float x = 0.f;
            switch (var) {
            case GEO_VAR_U: x = s.u[q]; break;
            case GEO_VAR_S: x = s.s[q]; break;
            case GEO_VAR_T: x = s.t[q]; break;
            case GEO_VAR_W1:
            case GEO_VAR_W2: {
                const float2 w = *w_pair(wp, N, pl >> 1, q);
                x = (pl & 1) ? w.y : w.x;
            } break;
            case GEO_VAR_Y1:
            case GEO_VAR_Y2: {
                const float2 y = ld2(yp + q);
                x = pl ? y.y : y.x;
            } break;
            case GEO_VAR_Y3: x = ld(s.y3 + q); break;
            default: x = y4_of(ld(s.y4 + q), a4); break;
            }
            out[g] = x;
        } else {
            switch (var) {
            case GEO_VAR_U: s.u[q] = in[q]; break;
            case GEO_VAR_S: s.s[q] = in[q]; break;
            case GEO_VAR_T: s.t[q] = in[q]; break;
            case GEO_VAR_W1:
            case GEO_VAR_W2:
                if ((pl & 1) == 0) *w_pair(wp, N, pl >> 1, q) = make_float2(in[g], in[g + N]);
                break;
            case GEO_VAR_Y1:
            case GEO_VAR_Y2:
                // both sides: sweep A never rewrites the masked entries
                if (pl == 0) {
                    const float2 y = make_float2(in[q], in[q + N]);
                    st2((var == GEO_VAR_Y1 ? s0.y1 : s0.y2) + q, y);
                    st2((var == GEO_VAR_Y1 ? s1.y1 : s1.y2) + q, y);
                }
                break;
            case GEO_VAR_Y3: st(s.y3 + q, in[q]); break;
            default: st(s.y4 + q, in[q]); break;
            }
        }
    }
}

// After a state load: y4 loaded as-is is read back with the factor 1, and
// the threshold predictions are dropped (the loaded state does not continue
// the previous run).
__global__ void k_state_loaded(DevScalars *sc, int var)
{
    if (threadIdx.x == 0) {
        if (var == GEO_VAR_Y4) sc->a4 = 1.0;
        for (int f = 0; f < 2; ++f) {
            sc->sel[f].win_on = 0u;
            sc->sel[f].tau_prev = 0.0;
            sc->sel[f].tau_prev2 = 0.0;
            sc->sel[f].tau_prev3 = 0.0;
            sc->sel[f].done = 1u;
        }
        sc->zstore = 1u;
        sc->calm = 0u;
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
    s.w1 = (float2 *)(b + L.w1[p]);
    s.w2 = (float2 *)(b + L.w2[p]);
    s.y1 = (typename Side<DT>::P *)(b + L.y1[p]);
    s.y2 = (typename Side<DT>::P *)(b + L.y2[p]);
    s.y3 = (DT *)(b + L.y3[p]);
    s.y4 = (DT *)(b + L.y4[p]);
    return s;
}

int grid_for(int64_t n)
{
    int64_t b = (n + NPT - 1) / NPT;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

// Resident blocks of sweep A on this device (queried once per process and
// storage type).
template <typename DT>
int resident_grid()
{
    // computed once per process (thread-safe initialisation of a local static)
    static const int cached = [] {
        int dev = 0, cus = 256, p0 = 1, p1 = 1;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
        }
        // the smaller occupancy of the tile shapes in use
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&p0, k_sweep_a<DT, 0>, NT, 0) != hipSuccess || p0 < 1)
            p0 = 1;
        p1 = p0;
        if constexpr (sizeof(DT) == 4)
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&p1, k_sweep_a<DT, 1>, NT, 0) != hipSuccess ||
                p1 < 1)
                p1 = 1;
        return cus * (p0 < p1 ? p0 : p1);
    }();
    return cached;
}

template <typename DT>
void cube_entry_t(CubeArgs<DT> *a, const Dims &d, const float *v, void *ws, const Layout &L,
                  double omega, double mu_lo, double mu_hi, int kc, int tile0, int b0, int *ntiles,
                  int *nb)
{
    char *b = (char *)ws;
    memset(a, 0, sizeof *a);
    CubeCommon &c = a->c;
    c.d = d;
    c.v = v;
    c.sc = (DevScalars *)(b + L.scalars);
    c.part = (double *)(b + L.partials);
    c.winpart = (double *)(b + L.winpart);
    c.hist = (Hist *)(b + L.hist);
    c.rec = (FbRec *)(b + L.rec);
    c.cand = (float *)(b + L.cand);
    c.zbuf = (float *)(b + L.zbuf);
    c.ccount = (uint32_t *)(b + L.ccount);
    const int shape = tile_shape(d.n1, d.n2, (int)sizeof(DT));
    c.g = sweep_grid(d.n1, d.n2, d.n3, band_chunk(d.n1, d.n2, d.n3, kc, sweep_a_grid(sizeof(DT), 1 << 30), shape),
                     shape);
    c.ntiles = c.g.blocks();
    c.capt = (int)(L.cap / c.ntiles);
    c.tile0 = tile0;
    {
        // strips of RB rows and CPT columns; never more blocks than the
        // partials hold
        const int64_t items = (int64_t)d.n3 * ((d.n1 + RB - 1) / RB) * (d.n2 / sweep_b_cpt(d.n2, (int)sizeof(DT)));
        const int pb = point_blocks(items);
        c.nb = pb < kSweepBBlocks ? pb : kSweepBBlocks;
    }
    c.b0 = b0;
    c.thr1 = (float)(omega * 0.25);
    c.zt_step = kStepT;
    c.mu_lo = (float)mu_lo;
    c.mu_hi = (float)mu_hi;
    a->side[0] = side_of<DT>(ws, L, 0);
    a->side[1] = side_of<DT>(ws, L, 1);
    a->y4p = (DT *)(b + L.y4p);
    for (int p = 0; p < 2; ++p) {
        c.bin[p][0] = a->side[p].s;
        c.bin[p][1] = a->side[p].t;
        c.bin[p][2] = a->side[p].y3;
        c.bin[p][3] = a->side[p].y4;
        c.bin[p][4] = a->y4p;
    }
    const size_t N = (size_t)d.plane;
    c.bin_bytes[0] = c.bin_bytes[1] = N * sizeof(float);
    c.bin_bytes[2] = c.bin_bytes[3] = c.bin_bytes[4] = N * sizeof(DT);
    *ntiles = c.ntiles;
    *nb = c.nb;
}

template <typename DT>
hipError_t slot_t(const void *table, const LaunchShape &sh, hipStream_t st, hipEvent_t *ev, int nev)
{
    const CubeArgs<DT> *cubes = (const CubeArgs<DT> *)table;
    const int stride = (int)sizeof(CubeArgs<DT>);
    if (nev >= 2) (void)hipEventRecord(ev[0], st);
    // one persistent launch per tile shape present (each takes the tiles of
    // its cubes)
    if (sh.shape_tiles[0] > 0)
        hipLaunchKernelGGL((k_sweep_a<DT, 0>), dim3(sh.shape_grid[0]), dim3(NT), 0, st, cubes, sh);
    if constexpr (sizeof(DT) == 4)  // BF16 duals use 8 x 128 tiles only
        if (sh.shape_tiles[1] > 0)
            hipLaunchKernelGGL((k_sweep_a<DT, 1>), dim3(sh.shape_grid[1]), dim3(NT), 0, st, cubes, sh);
    if (nev >= 2) (void)hipEventRecord(ev[1], st);
    hipError_t e = launch_select_window(table, stride, sh.ncubes, kPrefetchBlocks, st);
    for (int level = 0; level < 3 && e == hipSuccess; ++level)
        e = launch_fallback(table, (int)sizeof(DT), sh, level, st);
    if (e != hipSuccess) return e;
    if (nev >= 4) (void)hipEventRecord(ev[2], st);
    if (sh.b_kinds & 1)
        hipLaunchKernelGGL((k_sweep_b<DT, false>), dim3(sh.total_b), dim3(NPT), 0, st, cubes, sh);
    if (sh.b_kinds & 2)
        hipLaunchKernelGGL((k_sweep_b<DT, true>), dim3(sh.total_b), dim3(NPT), 0, st, cubes, sh);
    hipLaunchKernelGGL(k_finalize, dim3(sh.ncubes), dim3(NPT), 0, st, (const char *)table, stride);
    if (nev >= 4) (void)hipEventRecord(ev[3], st);
    return hipGetLastError();
}

}  // namespace

void cube_entry(CubeEntry *e, const Dims &d, const float *v, void *ws, const Layout &L, double omega,
                double mu_lo, double mu_hi, int kc, int tile0, int b0, int *ntiles, int *nb)
{
    if (L.dual_bytes == 2)
        cube_entry_t<bf16>(reinterpret_cast<CubeArgs<bf16> *>(e->bytes), d, v, ws, L, omega, mu_lo,
                           mu_hi, kc, tile0, b0, ntiles, nb);
    else
        cube_entry_t<float>(reinterpret_cast<CubeArgs<float> *>(e->bytes), d, v, ws, L, omega, mu_lo,
                            mu_hi, kc, tile0, b0, ntiles, nb);
}

// Persistent sweep A grid: resident blocks, at most one per tile, a multiple
// of the 8 XCDs when it is smaller than the tile count.
int sweep_a_grid(int dual_bytes, int total_tiles)
{
    int G = dual_bytes == 2 ? resident_grid<bf16>() : resident_grid<float>();
    if (G >= total_tiles) return total_tiles;
    return G >= 8 ? (G & ~7) : G;
}

hipError_t launch_slot(const void *table, int dual_bytes, const LaunchShape &sh, hipStream_t st,
                       hipEvent_t *ev, int nev)
{
    if (!ev) nev = 0;
    return dual_bytes == 2 ? slot_t<bf16>(table, sh, st, ev, nev) : slot_t<float>(table, sh, st, ev, nev);
}

hipError_t launch_finalize(const void *table, int stride, int ncubes, hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize, dim3(ncubes), dim3(NPT), 0, st, (const char *)table, stride);
    return hipGetLastError();
}

hipError_t launch_state_loaded(DevScalars *sc, int var, hipStream_t st)
{
    hipLaunchKernelGGL(k_state_loaded, dim3(1), dim3(64), 0, st, sc, var);
    return hipGetLastError();
}

hipError_t launch_init(const Dims &d, const float *v, void *ws, const Layout &L, double eps,
                       double tol, double alpha, double beta, hipStream_t st)
{
    DevScalars *sc = (DevScalars *)((char *)ws + L.scalars);
    if (L.dual_bytes == 2)
        hipLaunchKernelGGL(k_init<bf16>, dim3(grid_for(d.plane)), dim3(NPT), 0, st, d, v,
                           side_of<bf16>(ws, L, 0), side_of<bf16>(ws, L, 1), sc, eps, tol, alpha, beta);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(grid_for(d.plane)), dim3(NPT), 0, st, d, v,
                           side_of<float>(ws, L, 0), side_of<float>(ws, L, 1), sc, eps, tol, alpha,
                           beta);
    return hipGetLastError();
}

hipError_t launch_begin_call(void *ws, const Layout &L, double tol, double alpha, double beta,
                             int call_limit, hipStream_t st)
{
    DevScalars *sc = (DevScalars *)((char *)ws + L.scalars);
    hipLaunchKernelGGL(k_begin_call, dim3(1), dim3(64), 0, st, sc, tol, alpha, beta,
                       (uint32_t)call_limit);
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
        hipLaunchKernelGGL(k_state_io<bf16>, dim3(grid), dim3(NPT), 0, st, d, side_of<bf16>(ws, L, 0),
                           side_of<bf16>(ws, L, 1), sc, var, v, out, in);
    else
        hipLaunchKernelGGL(k_state_io<float>, dim3(grid), dim3(NPT), 0, st, d,
                           side_of<float>(ws, L, 0), side_of<float>(ws, L, 1), sc, var, v, out, in);
    if (in) hipLaunchKernelGGL(k_state_loaded, dim3(1), dim3(64), 0, st, sc, var);
    return hipGetLastError();
}

}  // namespace geo
