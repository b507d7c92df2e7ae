// Exact l1-ball thresholds whose predicted window missed, found inside the
// same launch slot: three histogram passes over the field (the radix levels
// of radix.hpp), one launch each, between the window search and sweep B.
//
// Each launch is a no-op (its blocks read one flag of the launch and leave)
// unless the window search of this slot left a field of some working cube
// pending. The blocks then split the voxels of the cubes with a pending
// field evenly, read z_s and z_t where sweep A stored them in this
// iteration, or else evaluate them from the state exactly as sweep A does
// (the same rounding operations, so the values are bit-identical), keep the
// values whose higher bits match the bins the earlier levels chose, and add
// them to LDS histograms that are flushed into the cube's global histogram
// of the level with integer atomics (order-free, exact). The last block to
// finish a cube (a counter, no waiting) reads the level back.
#include "radix.hpp"

namespace geo {

namespace {

// One 1024-thread block per CU: the blocks' atomics on a common bin of the
// global histogram are performed one after another, so fewer, larger blocks
// shorten that chain.
constexpr int kFbThreads = 1024;
constexpr int kFbUnroll = 4;    // voxels per thread in flight at once (from the state)
constexpr int kFbUnrollZ = 16;  // and from stored z (one load per field and voxel)

// Blocks of a pass whose voxel range [W b / G, W (b + 1) / G) meets the
// work range [c0, c1) of a cube (empty ranges inside it count too): the
// first is the smallest b with W (b + 1) / G > c0, the last the largest b
// with W b / G < c1 (integer divisions).
__device__ __forceinline__ int blocks_meeting(int64_t W, int G, int64_t c0, int64_t c1)
{
    const int64_t first = (G * (c0 + 1) + W - 1) / W - 1;
    const int64_t last = (G * c1 + W - 1) / W - 1;
    return (int)(last - first + 1);
}

// One pass: the histogram of radix level `level` of every field whose
// window missed and whose search reached this level. The last block to
// finish a cube's share reads that cube's histograms back (the level's
// bin, or the threshold when the level ends the search) into the field's
// record of the level, which the next pass, sweep B and the finalize read.
// A pass writes nothing that its own blocks read at their start (a block
// may start after another cube's last block is done), so every block sees
// the same work.
template <typename DT>
__global__ __launch_bounds__(kFbThreads) void k_fb_hist(const CubeArgs<DT> *__restrict__ cubes,
                                                         LaunchShape sh, int level,
                                                         const uint32_t *pending)
{
    if (*pending == 0u) return;  // no window missed in this slot
    __shared__ uint32_t hc[2][kHistBins];
    __shared__ unsigned long long hm[2][kHistBins];
    __shared__ int64_t seg0[kMaxBatch + 1];  // first work index of each cube
    __shared__ uint32_t fmask[kMaxBatch];    // fields of each cube at this level
    __shared__ RadixPick pick_out;
    __shared__ int last;
    static_assert(kMaxBatch <= 64, "one wavefront scans the cubes");
    const int tid = threadIdx.x;
    if (tid < 64) {
        const int c = tid;
        uint32_t m = 0u;
        int64_t n = 0;
        if (c < sh.ncubes) {
            const DevScalars *sc = cubes[c].c.sc;
            // fields still searching at this level: the window search and the
            // earlier passes decided it (nothing this pass writes is read here)
            if (!idle(sc))
                for (int f = 0; f < 2; ++f)
                    if (!sc->sel[f].done && (level == 0 || !cubes[c].c.rec[(level - 1) * 2 + f].done))
                        m |= 1u << f;
            if (m) n = cubes[c].c.d.plane;
        }
        int64_t x = n;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o, 64);
            if (c >= o) x += y;
        }
        if (c < sh.ncubes) {
            seg0[c + 1] = x;
            fmask[c] = m;
        }
        if (c == 0) seg0[0] = 0;
    }
    __syncthreads();
    const int64_t W = seg0[sh.ncubes];
    if (W == 0) return;
    const int G = (int)gridDim.x;
    const int64_t lo = W * (int64_t)blockIdx.x / G, hi = W * (int64_t)(blockIdx.x + 1) / G;
    const int shift = lvl_shift(level), pshift = shift + (level == 0 ? 11 : 10);
    const uint32_t bmask = (uint32_t)lvl_bins(level) - 1u;
    for (int c = 0; c < sh.ncubes; ++c) {
        const int64_t c0 = seg0[c], c1 = seg0[c + 1];
        if (c0 == c1 || !(lo < c1 && hi > c0)) continue;  // the block takes no part in cube c
        const CubeArgs<DT> &a = cubes[c];
        DevScalars *sc = a.c.sc;
        const uint32_t m = fmask[c];
        const bool act0 = m & 1u, act1 = m & 2u;
        const FbRec *rec = a.c.rec;
        const uint32_t pre0 = level ? rec[(level - 1) * 2].prefix : 0u;
        const uint32_t pre1 = level ? rec[(level - 1) * 2 + 1].prefix : 0u;
        for (int b = tid; b < 2 * kHistBins; b += kFbThreads) {
            hc[b / kHistBins][b % kHistBins] = 0u;
            hm[b / kHistBins][b % kHistBins] = 0ull;
        }
        __syncthreads();
        {
            const Dims d = a.c.d;
            const int n1 = d.n1, n2 = d.n2;
            const int par = (int)(sc->iter & 1u);
            const Side<DT> src = a.side[par];
            const float a4 = (float)sc->a4, gt = a.c.zt_step;
            // z as sweep A stored it in this iteration, or evaluated again
            const float *zb = sc->zstore ? a.c.zbuf : nullptr;
            const uint32_t N = (uint32_t)d.plane;
            const uint32_t q0 = (uint32_t)((lo > c0 ? lo : c0) - c0), q1 = (uint32_t)((hi < c1 ? hi : c1) - c0);
            auto add = [&](int f, uint32_t pre, float z) {
                const uint32_t p = abs_bits(z);
                if (level > 0 && (p >> pshift) != pre) return;
                const uint32_t b = (p >> shift) & bmask;
                atomicAdd(&hc[f][b], 1u);
                atomicAdd(&hm[f][b], (unsigned long long)significand(p));
            };
            if (zb) {
                for (uint32_t q = q0 + (uint32_t)tid; q < q1; q += kFbUnrollZ * kFbThreads) {
                    float z0[kFbUnrollZ], z1[kFbUnrollZ];
#pragma unroll
                    for (int u = 0; u < kFbUnrollZ; ++u) {
                        const uint32_t x = q + (uint32_t)(u * kFbThreads);
                        z0[u] = z1[u] = 0.f;
                        if (x < q1) {
                            if (act0) z0[u] = zb[x];
                            if (act1) z1[u] = zb[N + x];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kFbUnrollZ; ++u) {
                        if (q + (uint32_t)(u * kFbThreads) >= q1) break;
                        if (act0) add(0, pre0, z0[u]);
                        if (act1) add(1, pre1, z1[u]);
                    }
                }
            } else
            for (uint32_t q = q0 + (uint32_t)tid; q < q1; q += kFbUnroll * kFbThreads) {
                // every load of kFbUnroll voxels first, then their bins
                float y4s[kFbUnroll], sv[kFbUnroll], tv[kFbUnroll], y3c[kFbUnroll], y3m[kFbUnroll];
#pragma unroll
                for (int u = 0; u < kFbUnroll; ++u) {
                    const uint32_t x = q + (uint32_t)(u * kFbThreads);
                    y4s[u] = sv[u] = tv[u] = y3c[u] = y3m[u] = 0.f;
                    if (x < q1) {
                        y4s[u] = ld(src.y4 + x);
                        if (act0) sv[u] = src.s[x];
                        if (act1) {
                            const int i = (int)((x / (uint32_t)n2) % (uint32_t)n1);
                            tv[u] = src.t[x];
                            if (i <= n1 - 2) y3c[u] = ld(src.y3 + x);
                            if (i >= 1) y3m[u] = ld(src.y3 + x - n2);
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < kFbUnroll; ++u) {
                    if (q + (uint32_t)(u * kFbThreads) >= q1) break;
                    const float y4 = y4_of(y4s[u], a4);
                    if (act0) add(0, pre0, zs_of(sv[u], y4));
                    if (act1) add(1, pre1, zt_of(tv[u], y3m[u], y3c[u], y4, gt));
                }
            }
        }
        __syncthreads();
        // The block's histograms go to the global ones with atomics of system
        // scope, performed beyond the XCD's L2 (visible to every XCD without
        // writing back any cache), and returning, so that the wait below
        // covers their completion; all of a thread's atomics go out before
        // their results are used. Then the block counts itself done with
        // the cube; the last one reads the histograms back.
        Hist *hist = a.c.hist;
        uint32_t seen = 0u;
        {
            constexpr int per = 2 * kHistBins / kFbThreads;
            uint32_t rc[per];
            unsigned long long rm[per];
#pragma unroll
            for (int k = 0; k < per; ++k) {
                const int b = tid + k * kFbThreads;
                const int f = b / kHistBins, bb = b % kHistBins;
                rc[k] = 0u;
                rm[k] = 0ull;
                if (hc[f][bb]) {
                    rc[k] = __hip_atomic_fetch_add(&hist[level * 2 + f].count[bb], hc[f][bb], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_SYSTEM);
                    rm[k] = __hip_atomic_fetch_add((unsigned long long *)&hist[level * 2 + f].msum[bb], hm[f][bb],
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
#pragma unroll
            for (int k = 0; k < per; ++k) seen |= rc[k] | (uint32_t)rm[k];
        }
        __builtin_amdgcn_s_waitcnt(0);  // this thread's atomics are done
        __syncthreads();
        uint32_t *counter = slot_flags(cubes, sh.ncubes) + kFbCounterWord + c;
        if (tid == 0) {
            const int nbk = blocks_meeting(W, G, c0, c1);
            const uint32_t done = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            last = done == (uint32_t)(nbk - 1) ? 1 : 0;
        }
        __syncthreads();
        // (the returned values are kept alive by a store no launch reaches:
        // a table holds at most kMaxBatch cubes)
        if (sh.ncubes > kMaxBatch && tid == 0) hc[0][0] = seen;
        if (last) {
            // acquire: drop cached copies so that the reads see every block's atomics
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            double *bs = reinterpret_cast<double *>(&hm[0][0]);
            uint32_t *bc = &hc[0][0];
            const int nb = lvl_bins(level);
            for (int f = 0; f < 2; ++f) {
                if (!(m >> f & 1u)) continue;
                RadixPick pk = {0.0, 0.0, 0.0, 0.0, 0u, level, 0};
                if (level > 0) {
                    const FbRec &pr = rec[(level - 1) * 2 + f];
                    pk.s_above = pr.s_above;
                    pk.c_above = pr.c_above;
                    pk.prefix = pr.prefix;
                }
                Hist &h = hist[level * 2 + f];
                for (int b = tid; b < nb; b += kFbThreads) {
                    // read where the atomics were performed
                    const uint32_t e = lvl_exponent(level, pk.prefix, b);
                    const unsigned long long ms = __hip_atomic_load((unsigned long long *)&h.msum[b], __ATOMIC_RELAXED,
                                                                    __HIP_MEMORY_SCOPE_SYSTEM);
                    bs[b] = (double)ms * bin_scale(e);
                    bc[b] = __hip_atomic_load((uint32_t *)&h.count[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                __syncthreads();
                if (tid < 64) {
                    radix_level_wave(bs, bc, sc->sel[f].radius, pk);
                    if (tid == 0) {
                        FbRec o;
                        o.tau = pk.tau;
                        o.s_above = pk.s_above;
                        o.c_above = pk.c_above;
                        o.dens = pk.dens;
                        o.prefix = pk.prefix;
                        o.done = pk.done ? 1u : 0u;
                        a.c.rec[level * 2 + f] = o;
                    }
                }
                __syncthreads();
            }
            if (tid == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        __syncthreads();  // the LDS histograms are reused by the next cube
    }
}

}  // namespace

// Persistent blocks of a fallback pass: one per compute unit.
int fallback_grid()
{
    static const int cached = [] {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
        }
        return cus;
    }();
    return cached;
}

hipError_t launch_fallback(const void *table, int dual_bytes, const LaunchShape &sh, int level,
                           hipStream_t st)
{
    const uint32_t *pending = slot_flags(table, sh.ncubes);
    if (dual_bytes == 2)
        hipLaunchKernelGGL(k_fb_hist<bf16>, dim3(sh.fb_grid), dim3(kFbThreads), 0, st,
                           (const CubeArgs<bf16> *)table, sh, level, pending);
    else
        hipLaunchKernelGGL(k_fb_hist<float>, dim3(sh.fb_grid), dim3(kFbThreads), 0, st,
                           (const CubeArgs<float> *)table, sh, level, pending);
    return hipGetLastError();
}

}  // namespace geo
